// Host runtime of the C ABI in include/fr.h: device mesh construction,
// operator tables, residual/tangent entry points, the restarted GMRES driver
// (optionally replayed as captured HIP graphs), pseudo-transient continuation
// with ESDIRK2, the smoothness indicator and the launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fr.h"
#include "frx_host.hpp"
#include "frx_krylov.hpp"
#include "frx_precond.hpp"

using namespace frx;


namespace {

thread_local std::string g_create_error;

struct HipErr {
  hipError_t e;
  const char* what;
};

#define FRX_TRY(call)                                  \
  do {                                                 \
    hipError_t _e = (call);                            \
    if (_e != hipSuccess) throw HipErr{_e, #call};     \
  } while (0)

struct StatusErr {
  fr_status st;
  std::string msg;
};

// ------------------------------------------------------------ operator tables
// Gauss-Legendre nodes by Newton's method on P_n, barycentric Lagrange
// weights, D by the barycentric differentiation formula, DG correction
// derivatives from the Legendre derivative identity
// (1 - x^2) P_k'(x) = k (P_{k-1}(x) - x P_k(x)).
void legendre_upto(int K, double x, double* P) {
  P[0] = 1.0;
  if (K > 0) P[1] = x;
  for (int k = 2; k <= K; ++k) P[k] = ((2.0 * k - 1.0) * x * P[k - 1] - (k - 1.0) * P[k - 2]) / k;
}

double legendre_d(int k, double x) {  // interior points only
  if (k == 0) return 0.0;
  double P[16];
  legendre_upto(k, x, P);
  return k * (P[k - 1] - x * P[k]) / (1.0 - x * x);
}

void gauss_nodes(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    // i-th root from the largest downwards, stored ascending
    double t = std::cos(M_PI * (4.0 * i + 3.0) / (4.0 * n + 2.0));
    for (int it = 0; it < 64; ++it) {
      double P[16];
      legendre_upto(n, t, P);
      const double dp = n * (P[n - 1] - t * P[n]) / (1.0 - t * t);
      const double step = P[n] / dp;
      t -= step;
      if (std::fabs(step) <= 1e-17) break;
    }
    const double dp = legendre_d(n, t);
    x[n - 1 - i] = t;
    w[n - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

struct Nodes {
  int n;
  double x[NMAX], w[NMAX], lam[NMAX];
};

Nodes make_nodes(int n) {
  Nodes N;
  N.n = n;
  gauss_nodes(n, N.x, N.w);
  for (int j = 0; j < n; ++j) {
    double p = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != j) p *= (N.x[j] - N.x[m]);
    N.lam[j] = 1.0 / p;
  }
  return N;
}

// l_j(t) for every j (barycentric form; t may coincide with a node)
void lagrange_at(const Nodes& N, double t, double* l) {
  for (int j = 0; j < N.n; ++j)
    if (t == N.x[j]) {
      for (int m = 0; m < N.n; ++m) l[m] = (m == j) ? 1.0 : 0.0;
      return;
    }
  double den = 0.0;
  for (int j = 0; j < N.n; ++j) den += N.lam[j] / (t - N.x[j]);
  for (int j = 0; j < N.n; ++j) l[j] = N.lam[j] / (t - N.x[j]) / den;
}

void build_tables(OpsTab<double>& T) {
  std::memset(&T, 0, sizeof(T));
  for (int n = 1; n <= NMAX; ++n) {
    Nodes N = make_nodes(n);
    const int p = n - 1;
    for (int k = 0; k < n; ++k) {
      T.x[n][k] = N.x[k];
      T.w[n][k] = N.w[k];
      double s = 0.0;
      for (int j = 0; j < n; ++j) {
        if (j == k) continue;
        const double d = (N.lam[j] / N.lam[k]) / (N.x[k] - N.x[j]);
        T.D[n][k][j] = d;
        s += d;
      }
      T.D[n][k][k] = -s;
      // g_L = (-1)^(p+1)/2 (P_{p+1} - P_p): right Radau polynomial, g_L(-1) = 1
      const double sg = (p % 2 == 0) ? -0.5 : 0.5;
      T.gL[n][k] = sg * (legendre_d(p + 1, N.x[k]) - legendre_d(p, N.x[k]));
      T.gR[n][k] = -sg * (legendre_d(p + 1, -N.x[k]) - legendre_d(p, -N.x[k]));
      double P[16];
      legendre_upto(n - 1, N.x[k], P);
      for (int m = 0; m < n; ++m) {
        T.V[n][k][m] = P[m];
        T.Vinv[n][m][k] = 0.5 * (2.0 * m + 1.0) * N.w[k] * P[m];
      }
    }
    double l[NMAX];
    lagrange_at(N, -1.0, l);
    for (int j = 0; j < n; ++j) T.lm[n][j] = l[j];
    lagrange_at(N, 1.0, l);
    for (int j = 0; j < n; ++j) T.lp[n][j] = l[j];
  }
  for (int nl = 2; nl <= NMAX; ++nl)
    for (int nh = nl + 1; nh <= NMAX; ++nh) {
      Nodes L = make_nodes(nl), H = make_nodes(nh);
      for (int A = 0; A < nh; ++A) {
        double l[NMAX];
        lagrange_at(L, H.x[A], l);
        for (int a = 0; a < nl; ++a) {
          T.I[nl - 2][nh - 2][A][a] = l[a];
          T.P[nl - 2][nh - 2][a][A] = H.w[A] * l[a] / L.w[a];
        }
      }
    }
}

template <class B, class S> void cast_tables(const OpsTab<S>& s, OpsTab<B>& d) {
  const S* ps = reinterpret_cast<const S*>(&s);
  B* pd = reinterpret_cast<B*>(&d);
  for (size_t i = 0; i < sizeof(s) / sizeof(S); ++i) pd[i] = (B)ps[i];
}

bool g_tables_uploaded[64] = {false};

void ensure_tables(int dev) {
  if (dev >= 0 && dev < 64 && g_tables_uploaded[dev]) return;
  std::unique_ptr<OpsTab<double>> td(new OpsTab<double>);
  std::unique_ptr<OpsTab<float>> tf(new OpsTab<float>);
  build_tables(*td);
  cast_tables<float, double>(*td, *tf);
  FRX_TRY(upload_tables_f64(*td, *tf));
  FRX_TRY(upload_tables_dual64(*td, *tf));
  FRX_TRY(upload_tables_dual32(*td, *tf));
  FRX_TRY(upload_tables_vjp(*td, *tf));
  if (dev >= 0 && dev < 64) g_tables_uploaded[dev] = true;
}

constexpr int NBLK = 512;  // multi-dot blocks
constexpr int GS_PARTS = 65536;  // partial sums of one fused Gram-Schmidt launch

}  // namespace

namespace frx {
size_t scalar_bytes(int sk) { return sk == SK_F64 ? 8 : (sk == SK_DUAL64 ? 16 : 8); }

// Default shapes: about 256 threads per block, LDS per block capped at 48 KB.
void default_shapes(MeshDev& M, int sk) {
  const size_t sb = scalar_bytes(sk);
  const size_t cap = 64 * 1024;
  for (ElemBucket& b : M.eb) {
    const int n = b.n, n3 = n * n * n;
    const int tv = trace_lds_vals(M.physics == 1, n, (int)sb);
    int e = std::max(1, 256 / n3);
    while (e > 1 && (size_t)e * tv * n3 * sb > cap) --e;
    b.epb_trace[sk] = e;
    e = std::max(1, 256 / n3);
    while (e > 1 && (size_t)e * (5 * n3 + 30 * n * n) * sb > cap) --e;
    b.epb_div[sk] = e;
  }
  for (FaceBucket& f : M.fb) {
    int e = std::max(1, 256 / (f.nh * f.nh));
    const size_t per = f.nl < f.nh ? (size_t)(20 * f.nl * f.nl + 10 * f.nh * f.nh) * sb : 0;
    while (e > 1 && (size_t)e * per > cap) --e;
    f.fpb[sk] = e;
  }
}
}  // namespace frx

// =============================================== scratch of fr_residual_noalloc
// Face-slot buffers of the float64 residual for callers that cannot allocate:
// a file-scope device array (every GPU the library runs on holds its own copy
// until the process ends).  Host code never uses the array's name as an
// address: fr_create looks up each device's copy with hipGetSymbolAddress,
// with that device current, and keeps the pointer.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device -> address of its copy of `scratch`

// The address of `scratch` on device `dev`, which must be current.
void* scratch_on_device(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* p = nullptr;
  FRX_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw StatusErr{FR_E_HIP, "hipGetSymbolAddress returned no address for the static scratch"};
  g_scratch_ptr[dev] = p;
  return p;
}
}  // namespace

// ===================================================================== context
struct GraphKey {
  int mode, prec, j0, j1;  // Arnoldi iterations j0 .. j1 - 1 of a cycle (any length <= the reserved restart)
  bool operator<(const GraphKey& o) const {
    return std::tie(mode, prec, j0, j1) < std::tie(o.mode, o.prec, o.j0, o.j1);
  }
};
// Captured Arnoldi graphs, all instantiated by fr_reserve for the reserved
// restart M: "heads" cover iterations [0, h) for h in {3, 6, 12} below M,
// and h = M when M <= 12; "chunks" cover [3i, min(3i + 3, M)).  (Longer heads
// would save a few host round trips per long cycle, and doubled the capture
// work of every new context, which the p-adaptation makes at every step.)
// A cycle replays the largest
// head not above the iterations that the previous cycle of the same (mode,
// precision) needed, then chunks.  Between two graphs the host reads the
// device's converged flag, so a converged cycle stops early instead of
// replaying skipped kernels up to its end.  The cycle length, the shift and
// the finite-difference step are read from device memory, so one graph set
// serves every restart <= M and every step size.
constexpr int ARNOLDI_CHUNK = 3;
constexpr int ARNOLDI_HEAD_MAX = 12;
std::vector<int> arnoldi_heads(int M) {
  std::vector<int> h;
  for (int k = ARNOLDI_CHUNK; k < M && k <= ARNOLDI_HEAD_MAX; k *= 2) h.push_back(k);
  if (M <= ARNOLDI_HEAD_MAX) h.push_back(M);
  return h;
}
// graph-set bits of fr_reserve for (jv mode, precision)
inline int graph_bit(int mode, int prec) {
  return mode == FR_JV_EXACT ? (prec == FR_F32 ? FR_GRAPHS_F32_EXACT : FR_GRAPHS_F64_EXACT)
                             : (mode == FR_JV_FD ? FR_GRAPHS_F64_FD : FR_GRAPHS_F64_FD_SCALED);
}

// Device memory of the contexts comes from, and goes back to, a cache of
// freed blocks per device.  A p-adaptation replaces a context by one of
// nearly the same sizes (Krylov basis, face slots, stage vectors), so the
// new context takes the blocks the old one returned instead of unmapping and
// mapping hundreds of MB.  A request takes the smallest cached block of at
// least its size if that block is at most 1/8 larger; a miss allocates, and
// an allocation failure empties the device's cache and tries once more.
// Returned blocks beyond 16 GB of cache per device are freed.  fr_trim
// empties the caches.  The same holds for the two small pinned host buffers
// of every context.
namespace {
struct BlockCache {
  std::mutex mu;
  std::map<int, std::multimap<size_t, void*>> dev_free;  // device -> (size, block)
  std::map<int, size_t> dev_bytes;
  std::vector<void*> host_free;                          // pinned host blocks of HOST_BLOCK bytes
};
BlockCache& block_cache() {
  static BlockCache* c = new BlockCache;  // never destroyed: blocks may be returned at process exit
  return *c;
}
constexpr size_t CACHE_CAP = 16ull << 30;
constexpr size_t HOST_BLOCK = 64 * sizeof(double);

void* cache_take(int dev, size_t bytes, size_t* got) {
  BlockCache& C = block_cache();
  std::lock_guard<std::mutex> lock(C.mu);
  auto& m = C.dev_free[dev];
  auto it = m.lower_bound(bytes);
  if (it == m.end() || it->first > bytes + bytes / 8) return nullptr;
  void* p = it->second;
  *got = it->first;
  C.dev_bytes[dev] -= it->first;
  m.erase(it);
  return p;
}
void cache_give(int dev, void* p, size_t bytes) {
  BlockCache& C = block_cache();
  {
    std::lock_guard<std::mutex> lock(C.mu);
    if (C.dev_bytes[dev] + bytes <= CACHE_CAP) {
      C.dev_free[dev].emplace(bytes, p);
      C.dev_bytes[dev] += bytes;
      return;
    }
  }
  (void)hipFree(p);
}
void cache_empty(int dev) {
  BlockCache& C = block_cache();
  std::lock_guard<std::mutex> lock(C.mu);
  for (auto& kv : C.dev_free[dev]) (void)hipFree(kv.second);
  C.dev_free[dev].clear();
  C.dev_bytes[dev] = 0;
}
void* host_take() {
  BlockCache& C = block_cache();
  {
    std::lock_guard<std::mutex> lock(C.mu);
    if (!C.host_free.empty()) {
      void* p = C.host_free.back();
      C.host_free.pop_back();
      return p;
    }
  }
  void* p = nullptr;
  FRX_TRY(hipHostMalloc(&p, HOST_BLOCK, 0));
  return p;
}
void host_give(void* p) {
  if (!p) return;
  BlockCache& C = block_cache();
  std::lock_guard<std::mutex> lock(C.mu);
  C.host_free.push_back(p);
}
}  // namespace

struct fr_ctx_s {
  MeshDev M;
  int dev = 0;
  long ndof = 0;
  std::string err;
  std::vector<int8_t> p;
  std::vector<int64_t> sp_off_h;
  std::vector<int> fp_off_h;      // first face slot of each element
  std::vector<std::pair<void*, size_t>> allocs;  // device blocks and their sizes (from the block cache)
  hipStream_t cap = nullptr;  // private stream for graph capture
  // scratch for fr_jvp / operators
  double* t0 = nullptr;   // ndof
  double* t1 = nullptr;   // ndof
  double* t2 = nullptr;   // ndof
  float* uf = nullptr;    // ndof float copy of a state
  double* part = nullptr; // multi-dot partials [(mmax+2) x NBLK]
  double* sc = nullptr;   // small device scalars
  int* ist = nullptr;     // small device ints
  double* hpin = nullptr; // pinned host scalars
  int* ipin = nullptr;
  // Krylov workspace
  int m_alloc = -1;      // largest cycle the Krylov workspace holds
  void* Vb = nullptr;     // (m+1) x ndof basis
  void* wv = nullptr;     // ndof work vector (basis type)
  void* xv = nullptr;     // ndof basis-type copy of x
  double* Ulin = nullptr; // linearisation point
  double* Fb = nullptr;   // right-hand side
  double* R0 = nullptr;   // R(Ulin) for finite differences
  double* Up = nullptr;
  double* R1 = nullptr;
  double* rb = nullptr;   // restart residual
  double* H = nullptr;    // Hessenberg etc. (one block)
  float* sigf = nullptr;  // float copy of the shift
  std::map<GraphKey, hipGraphExec_t> graphs;
  int graph_sets = 0;  // FR_GRAPHS_* bits instantiated by fr_reserve
  std::map<std::pair<int, int>, int> cycle_iters;  // (mode, precision) -> iterations of the last cycle
  // fused plans: element ranges per degree, face ranges per code, chosen items
  // per tile per (scalar kind, stage, code) (absent: the default), table sizes
  std::map<int, std::pair<int, int>> erange;
  std::vector<std::tuple<int, int, int, int>> frange;
  std::map<int, int> shape[SK_COUNT][3];
  int plan_cap[3] = {0, 0, 0};
  // ESDIRK workspace
  double* es = nullptr;   // 8 x ndof
  // VJP workspace
  void* vjpw = nullptr;
  // this device's copy of the static scratch of fr_residual_noalloc
  void* scratch_dev = nullptr;
  // element-Jacobi preconditioner (section 2.3): storage made by fr_reserve
  // in one precision, built by fr_precond_build or at the start of a step
  void* pc_blocks = nullptr;   // dense blocks, column-major, [sum_e pc_block_size(N_e)] of pc_prec
  int pc_prec = -1;            // FR_F64 / FR_F32 storage, -1: none
  bool pc_built = false;
  bool pc_half = false;        // the built inverse is kept as float16 of sigma times it (float32 storage)
  double* pc_isig = nullptr;   // device: 1 / sigma of the last build
  int* pc_piv = nullptr;       // [sum_e N_e]
  int4* pc_recs = nullptr;     // [E] (e, first solution point, n, 0)
  long* pc_boff = nullptr;     // [E]
  int* pc_poff = nullptr;      // [E]
  int* pc_flag = nullptr;      // singular block met by the factorisation
  std::vector<int4*> pc_crecs; // per colour: records of its elements
  std::vector<int*> pc_cidx;   // per colour: their element ids
  std::vector<int> pc_ccount;
  int pc_nmax = 0;             // largest block order
  // per colour and n: the fused subset of the colour's elements of size >= n
  // (the elements that a column j < 5 n^3 seeds), null entries where no
  // element is that large
  std::vector<std::array<std::unique_ptr<FusedSubset>, NMAX + 1>> pc_sub;  // built by fr_reserve
  std::vector<int> pc_colour;  // colour of every element
  std::vector<int4> faces_h;   // host copy of the concatenated face list (ranges in frange)

  void* dalloc(size_t bytes) {
    bytes = (std::max<size_t>(bytes, 8) + 255) / 256 * 256;
    size_t got = 0;
    void* p = cache_take(dev, bytes, &got);
    if (!p) {
      got = bytes;
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        cache_empty(dev);
        e = hipMalloc(&p, bytes);
      }
      if (e != hipSuccess) throw StatusErr{FR_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
    }
    allocs.emplace_back(p, got);
    return p;
  }
  // (callers synchronise the device before they free: the block may be
  // handed to another context at once)
  void dfree(void* p) {
    if (!p) return;
    auto it = std::find_if(allocs.begin(), allocs.end(), [&](const std::pair<void*, size_t>& a) { return a.first == p; });
    if (it == allocs.end()) return;
    cache_give(dev, it->first, it->second);
    allocs.erase(it);
  }
  ~fr_ctx_s() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto& a : allocs) cache_give(dev, a.first, a.second);
    host_give(hpin);
    host_give(ipin);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

namespace {

fr_status fail(fr_ctx c, fr_status st, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_error = msg;
  return st;
}

template <class F> fr_status guarded(fr_ctx c, F&& f) {
  try {
    return f();
  } catch (const HipErr& h) {
    return fail(c, FR_E_HIP, std::string(h.what) + ": " + hipGetErrorString(h.e));
  } catch (const StatusErr& s) {
    return fail(c, s.st, s.msg);
  } catch (const std::bad_alloc&) {
    return fail(c, FR_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(c, FR_E_INVALID, "unexpected exception");
  }
}

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }
inline int grid_for(long n) { return (int)std::min<long>((n + KR_THREADS - 1) / KR_THREADS, 4096); }

// ------------------------------------------------------------- vector helpers
// dot(a, b) or |a|^2 (b == nullptr) into dst (device), deterministic
template <class TA>
void dot_to(fr_ctx c, const TA* a, const TA* b, double* dst, const int* done, hipStream_t s) {
  hipLaunchKernelGGL((k_multidot<TA, TA>), dim3(NBLK, 1), dim3(KR_THREADS), 0, s, b, (long)c->ndof, b ? 1 : 0, a,
                     (long)c->ndof, c->part, NBLK, done);
  FRX_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(KR_THREADS), 0, s, c->part, NBLK, dst, done);
  FRX_TRY(hipGetLastError());
}

double read_scalar(fr_ctx c, const double* d, hipStream_t s) {
  FRX_TRY(hipMemcpyAsync(c->hpin, d, sizeof(double), hipMemcpyDeviceToHost, s));
  FRX_TRY(hipStreamSynchronize(s));
  return c->hpin[0];
}

double norm2(fr_ctx c, const double* a, hipStream_t s) {
  dot_to<double>(c, a, nullptr, c->sc + 15, nullptr, s);
  return std::sqrt(read_scalar(c, c->sc + 15, s));
}

void lincomb(fr_ctx c, double* out, double c0, const double* x0, double c1 = 0, const double* x1 = nullptr,
             double c2 = 0, const double* x2 = nullptr, double c3 = 0, const double* x3 = nullptr,
             hipStream_t s = nullptr) {
  hipLaunchKernelGGL(k_lincomb, dim3(grid_for(c->ndof)), dim3(KR_THREADS), 0, s, out, (long)c->ndof, c0, x0, c1, x1,
                     c2, x2, c3, x3);
  FRX_TRY(hipGetLastError());
}

void check_flag(fr_ctx c, hipStream_t s) {
  FRX_TRY(hipMemcpyAsync(c->ipin, c->M.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  FRX_TRY(hipStreamSynchronize(s));
  if (c->ipin[0]) {
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, c->M.flag, 0);
    throw StatusErr{FR_E_NONPHYSICAL, "non-physical state (rho <= 0 or p <= 0) met in the residual"};
  }
}

// --------------------------------------------------------- Krylov workspace
// Device scalars: sc[0..5] GMRES (see GmresDev), sc[6] sigma, sc[8..] misc,
// sc[15] norm scratch; h1 = sc + 32, h2 = h1 + (mmax+1), nrm = h2 + (mmax+1).
void drop_graphs(fr_ctx c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

// Sized for cycles of up to m iterations; called by fr_create (m = 1) and
// fr_reserve only, never by a solver call.
void ensure_krylov(fr_ctx c, int m) {
  if (c->m_alloc >= m) return;
  const int mm = std::max(m, c->m_alloc);
  // graphs reference the old buffers
  drop_graphs(c);
  for (void* p : {c->Vb, c->wv, c->xv, (void*)c->H, (void*)c->part, (void*)c->sc, (void*)c->ist}) c->dfree(p);
  const size_t vb = 8;  // basis storage sized for float64 (float32 uses half)
  c->Vb = c->dalloc((size_t)(mm + 1) * c->ndof * vb);
  c->wv = c->dalloc((size_t)c->ndof * vb);
  c->xv = c->dalloc((size_t)c->ndof * vb);
  c->H = (double*)c->dalloc(sizeof(double) * ((mm + 1) * mm + 4 * (mm + 1)));
  c->part = (double*)c->dalloc(sizeof(double) * std::max<size_t>((size_t)(mm + 2) * NBLK, GS_PARTS));
  c->sc = (double*)c->dalloc(sizeof(double) * (64 + 3 * (mm + 2)));
  c->ist = (int*)c->dalloc(sizeof(int) * 16);
  FRX_TRY(hipMemset(c->ist, 0, sizeof(int) * 16));
  if (!c->Ulin) {
    c->Ulin = (double*)c->dalloc(sizeof(double) * c->ndof);
    c->Fb = (double*)c->dalloc(sizeof(double) * c->ndof);
    c->R0 = (double*)c->dalloc(sizeof(double) * c->ndof);
    c->Up = (double*)c->dalloc(sizeof(double) * c->ndof);
    c->R1 = (double*)c->dalloc(sizeof(double) * c->ndof);
    c->rb = (double*)c->dalloc(sizeof(double) * c->ndof);
    c->sigf = (float*)c->dalloc(sizeof(float) * 4);
  }
  c->m_alloc = mm;
}

GmresDev gdev(fr_ctx c) {
  GmresDev G;
  const int m = c->m_alloc;
  G.m = m;
  G.H = c->H;
  G.cs = c->H + (size_t)(m + 1) * m;
  G.sn = G.cs + (m + 1);
  G.g = G.sn + (m + 1);
  G.y = G.g + (m + 1);
  G.part = c->part;
  G.hbuf = c->sc + 32;
  G.sc = c->sc;
  G.ist = c->ist;
  G.nblk = NBLK;
  return G;
}

// Element-Jacobi preconditioner (apply; the build follows the Arnoldi code)
PcDev pc_dev(fr_ctx c) { return PcDev{c->pc_recs, c->pc_boff, c->pc_poff}; }

// x <- P^{-1} x (if the preconditioner is switched on: ist[5] on the device);
// nothing when the context has no preconditioner storage
template <class TV>
void pc_apply(fr_ctx c, TV* x, const int* done, hipStream_t s) {
  if (!c->pc_blocks) return;
  const int* on = c->ist + 5;  // 0 off, 1 stored inverse, 2 its float16 copy (chosen on the device)
  if (c->pc_prec == FR_F64)
    hipLaunchKernelGGL((k_pc_apply<TV, double>), dim3(c->M.E), dim3(256), 0, s, x, c->M.nsp,
                       (const double*)c->pc_blocks, pc_dev(c), (const int*)c->pc_piv, on, done,
                       (const double*)c->pc_isig);
  else
    hipLaunchKernelGGL((k_pc_apply<TV, float>), dim3(c->M.E), dim3(256), 0, s, x, c->M.nsp,
                       (const float*)c->pc_blocks, pc_dev(c), (const int*)c->pc_piv, on, done,
                       (const double*)c->pc_isig);
  FRX_TRY(hipGetLastError());
}

// The GMRES operator A x = sigma x - J(Ulin) x (sigma in sc[6], float copy in
// sigf) applied to `in` (basis type) into `out` (basis type).
template <class TV>
void apply_A(fr_ctx c, int mode, const TV* in, TV* out, const int* done, hipStream_t s) {
  const MeshDev& M = c->M;
  if (mode == FR_JV_EXACT) {
    if constexpr (sizeof(TV) == 8) {
      ResCall<double> rc;
      rc.U = c->Ulin;
      rc.V = (const double*)in;
      rc.out = (double*)out;
      rc.in2 = (const double*)in;
      rc.alpha_dev = c->sc + 6;
      rc.beta = -1.0;
      rc.skip = done;
      FRX_TRY(launch_residual_dual64(M, rc, s));
    } else {
      ResCall<float> rc;
      rc.U = c->uf;
      rc.V = (const float*)in;
      rc.out = (float*)out;
      rc.in2 = (const float*)in;
      rc.alpha_dev = c->sigf;
      rc.beta = -1.0f;
      rc.skip = done;
      FRX_TRY(launch_residual_dual32(M, rc, s));
    }
  } else {
    double* nrm = c->sc + 8;
    hipLaunchKernelGGL((k_multidot<TV, TV>), dim3(NBLK, 1), dim3(KR_THREADS), 0, s, (const TV*)nullptr,
                       (long)c->ndof, 0, in, (long)c->ndof, c->part, NBLK, done);
    FRX_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(KR_THREADS), 0, s, c->part, NBLK, nrm, done);
    FRX_TRY(hipGetLastError());
    hipLaunchKernelGGL((k_fd_perturb<TV>), dim3(grid_for(c->ndof)), dim3(KR_THREADS), 0, s, c->Ulin, in, nrm,
                       (const double*)(c->sc + 7), c->Up, (long)c->ndof, done);
    FRX_TRY(hipGetLastError());
    ResCall<double> rc;
    rc.U = c->Up;
    rc.out = c->R1;
    rc.skip = done;
    FRX_TRY(launch_residual_f64(M, rc, s));
    hipLaunchKernelGGL((k_fd_combine<TV, TV>), dim3(grid_for(c->ndof)), dim3(KR_THREADS), 0, s, in, c->R1, c->R0,
                       nrm, (const double*)(c->sc + 7), c->sc + 6, out, (long)c->ndof, done);
    FRX_TRY(hipGetLastError());
  }
}

// CGS2 for nv <= 32 basis vectors with the fused kernels: dots (h1), update
// fused with the second dots (h2), update fused with the norm and the Givens
// step; the orthogonalised vector goes straight into its basis slot (scaled
// afterwards by 1/h_{j+1,j}).
template <class TV, int NV>
void gs_fused_n(fr_ctx c, const GmresDev& G, int j, double* h1, double* h2, double* nr, TV* vnext, const int* done,
                hipStream_t s) {
  const long n = c->ndof;
  const TV* V = (const TV*)c->Vb;
  TV* w = (TV*)c->wv;
  // blocks: 2048 (8 per CU); the update-and-dot pass keeps all NV basis values
  // of its rows in registers and gets what stays resident of it at once
  constexpr int nb0 = 2048, nb1 = NV <= 8 ? 2048 : (NV <= 16 ? 1024 : 512);
  static_assert(NV * nb0 <= GS_PARTS && NV * nb1 <= GS_PARTS, "partials");
  // (ist[6] set: one-pass classical Gram-Schmidt; the second pass is skipped
  // and its coefficients read as 0)
  const int* one = c->ist + 6;
  hipLaunchKernelGGL((k_gs<TV, NV, 0>), dim3(nb0), dim3(KR_THREADS), 0, s, V, n, (const double*)nullptr, w,
                     (TV*)nullptr, n, c->part, done, (const double*)nullptr, (const int*)nullptr);
  FRX_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_gs_reduce, dim3(NV), dim3(KR_THREADS), 0, s, (const double*)c->part, nb0, h1, 0, G, j,
                     (const double*)nullptr, (const double*)nullptr, done, (const int*)nullptr);
  FRX_TRY(hipGetLastError());
  hipLaunchKernelGGL((k_gs<TV, NV, 1>), dim3(nb1), dim3(KR_THREADS), 0, s, V, n, (const double*)h1, w,
                     (TV*)nullptr, n, c->part, done, (const double*)nullptr, one);
  FRX_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_gs_reduce, dim3(NV), dim3(KR_THREADS), 0, s, (const double*)c->part, nb1, h2, 0, G, j,
                     (const double*)nullptr, (const double*)nullptr, done, one);
  FRX_TRY(hipGetLastError());
  hipLaunchKernelGGL((k_gs<TV, NV, 2>), dim3(nb0), dim3(KR_THREADS), 0, s, V, n, (const double*)h2, w, vnext, n,
                     c->part, done, (const double*)h1, one);
  FRX_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_gs_reduce, dim3(1), dim3(KR_THREADS), 0, s, (const double*)c->part, nb0, nr, 1, G, j,
                     (const double*)h1, (const double*)h2, done, (const int*)nullptr);
  FRX_TRY(hipGetLastError());
}

template <class TV, int NV = 1>
void gs_fused(fr_ctx c, const GmresDev& G, int j, double* h1, double* h2, double* nr, TV* vnext, const int* done,
              hipStream_t s) {
  if constexpr (NV <= 32) {
    if (j + 1 == NV) return gs_fused_n<TV, NV>(c, G, j, h1, h2, nr, vnext, done, s);
    return gs_fused<TV, NV + 1>(c, G, j, h1, h2, nr, vnext, done, s);
  } else {
    throw StatusErr{FR_E_INVALID, "fused Gram-Schmidt takes at most 32 vectors"};
  }
}

// One Arnoldi iteration j with CGS2, or one-pass CGS when ist[6] is set (all
// kernels skip once *done is set).
template <class TV>
void arnoldi_step(fr_ctx c, int mode, int j, hipStream_t s) {
  GmresDev G = gdev(c);
  const int m = G.m;
  const long n = c->ndof;
  TV* V = (TV*)c->Vb;
  TV* w = (TV*)c->wv;
  const int* done = c->ist;
  double* h1 = c->sc + 32;
  double* h2 = h1 + (m + 1);
  double* nr = h2 + (m + 1);
  apply_A<TV>(c, mode, V + (size_t)j * n, w, done, s);
  pc_apply<TV>(c, w, done, s);  // left preconditioning (a no-op unless switched on)
  const int nv = j + 1;
  if (nv <= 32) {
    gs_fused<TV>(c, G, j, h1, h2, nr, V + (size_t)(j + 1) * n, done, s);
    hipLaunchKernelGGL((k_scale_inplace<TV>), dim3(grid_for(n)), dim3(KR_THREADS), 0, s, V + (size_t)(j + 1) * n, n,
                       (const double*)(c->sc + 4), done);
    FRX_TRY(hipGetLastError());
    return;
  }
  const int gy = (nv + KR_VB - 1) / KR_VB;
  for (int pass = 0; pass < 2; ++pass) {
    double* h = pass ? h2 : h1;
    hipLaunchKernelGGL((k_multidot<TV, TV>), dim3(NBLK, gy), dim3(KR_THREADS), 0, s, (const TV*)V, n, nv,
                       (const TV*)w, n, c->part, NBLK, done);
    FRX_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_reduce, dim3(nv), dim3(KR_THREADS), 0, s, c->part, NBLK, h, done);
    FRX_TRY(hipGetLastError());
    hipLaunchKernelGGL((k_multiaxpy<TV, TV>), dim3(grid_for(n)), dim3(KR_THREADS), 0, s, (const TV*)V, n, nv,
                       (const double*)h, w, n, done);
    FRX_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL((k_multidot<TV, TV>), dim3(NBLK, 1), dim3(KR_THREADS), 0, s, (const TV*)nullptr, n, 0,
                     (const TV*)w, n, c->part, NBLK, done);
  FRX_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(KR_THREADS), 0, s, c->part, NBLK, nr, done);
  FRX_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_givens, dim3(1), dim3(1), 0, s, G, j, (const double*)h1, (const double*)h2,
                     (const double*)nr);
  FRX_TRY(hipGetLastError());
  hipLaunchKernelGGL((k_scale<TV, TV>), dim3(grid_for(n)), dim3(KR_THREADS), 0, s, (const TV*)w, V + (size_t)(j + 1) * n,
                     n, (const double*)(c->sc + 4), 0, done);
  FRX_TRY(hipGetLastError());
}

// Captures Arnoldi iterations [j0, j1) of (mode, TV) as a graph (fr_reserve).
template <class TV>
void capture_range(fr_ctx c, int mode, int j0, int j1) {
  if (!c->cap) FRX_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  hipGraph_t g;
  FRX_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  try {
    for (int j = j0; j < j1; ++j) arnoldi_step<TV>(c, mode, j, c->cap);
  } catch (...) {
    hipGraph_t tmp = nullptr;
    (void)hipStreamEndCapture(c->cap, &tmp);
    if (tmp) (void)hipGraphDestroy(tmp);
    throw;
  }
  FRX_TRY(hipStreamEndCapture(c->cap, &g));
  hipGraphExec_t ex;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  FRX_TRY(e);
  c->graphs[GraphKey{mode, (int)sizeof(TV), j0, j1}] = ex;
}

// Instantiates the heads and chunks of every graph set in c->graph_sets.
void instantiate_graphs(fr_ctx c) {
  drop_graphs(c);
  const int M = c->m_alloc;
  for (int bit : {FR_GRAPHS_F64_EXACT, FR_GRAPHS_F32_EXACT, FR_GRAPHS_F64_FD, FR_GRAPHS_F64_FD_SCALED}) {
    if (!(c->graph_sets & bit)) continue;
    const int mode = bit == FR_GRAPHS_F64_FD ? FR_JV_FD : (bit == FR_GRAPHS_F64_FD_SCALED ? FR_JV_FD_SCALED : FR_JV_EXACT);
    const bool f32 = bit == FR_GRAPHS_F32_EXACT;
    auto cap = [&](int j0, int j1) {
      if (f32) capture_range<float>(c, mode, j0, j1);
      else capture_range<double>(c, mode, j0, j1);
    };
    for (int h : arnoldi_heads(M)) cap(0, h);
    for (int j0 = 0; j0 < M; j0 += ARNOLDI_CHUNK) cap(j0, std::min(M, j0 + ARNOLDI_CHUNK));
  }
}

// One cycle of m <= M iterations (the length is in ist[4] on the device).
template <class TV>
void arnoldi_cycle(fr_ctx c, int mode, int m, bool use_graph, hipStream_t s) {
  if (!use_graph) {
    for (int j = 0; j < m; ++j) arnoldi_step<TV>(c, mode, j, s);
    return;
  }
  auto pit = c->cycle_iters.find({mode, (int)sizeof(TV)});
  const int prev = pit == c->cycle_iters.end() ? ARNOLDI_CHUNK : pit->second;
  int first = 0;
  for (int h : arnoldi_heads(c->m_alloc))
    if (first == 0 || h <= prev) first = h;  // the largest head <= prev, at least the smallest
  for (int j0 = 0; j0 < m;) {
    const int j1 = j0 == 0 ? first : std::min(c->m_alloc, j0 + ARNOLDI_CHUNK);
    auto it = c->graphs.find(GraphKey{mode, (int)sizeof(TV), j0, j1});
    if (it == c->graphs.end())
      throw StatusErr{FR_E_INVALID, "no reserved Arnoldi graph for this mode and precision (fr_reserve)"};
    FRX_TRY(hipGraphLaunch(it->second, s));
    if (j1 < m) {
      FRX_TRY(hipMemcpyAsync(c->ipin + 8, c->ist, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
      FRX_TRY(hipStreamSynchronize(s));
      if (c->ipin[8]) break;
    }
    j0 = j1;
  }
}

// ------------------------------------------------ element-Jacobi preconditioner
// Assembles the blocks sigma I - dR/dq(U)|_ee by coloured exact tangent
// products (the tangent in the storage precision: float64 duals on U, or
// float32 duals on a float32 copy of U), factors and inverts them.
void pc_build(fr_ctx c, const double* U, double sigma, hipStream_t s, bool half = false) {
  if (!c->pc_blocks) throw StatusErr{FR_E_INVALID, "no preconditioner storage (fr_reserve with FR_RESERVE_PRECOND_*)"};
  if (half && c->pc_prec != FR_F32) throw StatusErr{FR_E_INVALID, "a float16 inverse needs float32 storage"};
  c->pc_built = false;
  const long n = c->ndof;
  const bool f64 = c->pc_prec == FR_F64;
  if (!f64) {
    hipLaunchKernelGGL((k_cast<double, float>), dim3(grid_for(n)), dim3(KR_THREADS), 0, s, U, c->uf, n);
    FRX_TRY(hipGetLastError());
  }
  // seed and product vectors: t0 and t1 (n doubles hold n floats as well)
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(KR_THREADS), 0, s, c->t0, n, 0.0);
  FRX_TRY(hipGetLastError());
  for (size_t col = 0; col < c->pc_crecs.size(); ++col) {
    const int cnt = c->pc_ccount[col];
    if (!cnt) continue;
    // Traces of an element depend on its own U and v only.  The first product
    // of a colour traces every element; each later one traces the elements
    // seeded in the previous product (a superset of its own seeded elements):
    // that gives the newly seeded tangents and clears those of the elements
    // that dropped out, so every other element's slots keep their values and
    // a zero tangent.
    const FusedSubset* prev = nullptr;
    for (int j = 0; j <= c->pc_nmax; ++j) {
      const int jn = j < c->pc_nmax ? j : -1;  // the last pass only clears the seed
      if (f64)
        hipLaunchKernelGGL((k_pc_seed<double>), dim3((cnt + 255) / 256), dim3(256), 0, s, c->t0, c->M.nsp,
                           (const int4*)c->pc_crecs[col], cnt, j - 1, jn);
      else
        hipLaunchKernelGGL((k_pc_seed<float>), dim3((cnt + 255) / 256), dim3(256), 0, s, (float*)c->t0, c->M.nsp,
                           (const int4*)c->pc_crecs[col], cnt, j - 1, jn);
      FRX_TRY(hipGetLastError());
      if (jn < 0) break;
      // only the colour's elements of order N_e > j are seeded, and only
      // their rows are read: their faces and divergence suffice
      int nmin = 2;
      while (nmin < NMAX && 5 * nmin * nmin * nmin <= j) ++nmin;
      const FusedSubset* sub = c->M.fused ? c->pc_sub[col][nmin].get() : nullptr;
      if (c->M.fused && !sub) continue;  // no element of the colour has N_e > j
      if (f64) {
        ResCall<double> rc;
        rc.U = U;
        rc.V = c->t0;
        rc.out = c->t1;
        FRX_TRY(launch_residual_dual64(c->M, rc, s, sub, prev));
        hipLaunchKernelGGL((k_pc_extract<double, double>), dim3(cnt), dim3(256), 0, s, (const double*)c->t1,
                           c->M.nsp, (const int4*)c->pc_crecs[col], (const int*)c->pc_cidx[col], j, sigma,
                           (const long*)c->pc_boff, (double*)c->pc_blocks);
      } else {
        ResCall<float> rc;
        rc.U = c->uf;
        rc.V = (const float*)c->t0;
        rc.out = (float*)c->t1;
        FRX_TRY(launch_residual_dual32(c->M, rc, s, sub, prev));
        hipLaunchKernelGGL((k_pc_extract<float, float>), dim3(cnt), dim3(256), 0, s, (const float*)c->t1,
                           c->M.nsp, (const int4*)c->pc_crecs[col], (const int*)c->pc_cidx[col], j, sigma,
                           (const long*)c->pc_boff, (float*)c->pc_blocks);
      }
      FRX_TRY(hipGetLastError());
      prev = sub;
    }
  }
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, c->pc_flag, 0);
  // factorisation and inverse per degree bucket, with LDS for that order
  for (const ElemBucket& eb : c->M.eb) {
    if (!eb.count) continue;
    const int N = 5 * eb.n * eb.n * eb.n;
    if (f64) {
      FRX_TRY(pc_lu_launch<double>((double*)c->pc_blocks, pc_dev(c), (const int*)eb.elems, eb.count, N, c->pc_piv,
                                   c->pc_flag, s));
      FRX_TRY(pc_inv_launch<double>((double*)c->pc_blocks, pc_dev(c), (const int*)eb.elems, eb.count, N, s));
    } else {
      FRX_TRY(pc_lu_launch<float>((float*)c->pc_blocks, pc_dev(c), (const int*)eb.elems, eb.count, N, c->pc_piv,
                                  c->pc_flag, s));
      FRX_TRY(pc_inv_launch<float>((float*)c->pc_blocks, pc_dev(c), (const int*)eb.elems, eb.count, N, s));
      if (half) {
        FRX_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_pc_to_half, dim3(eb.count), dim3(256), 0, s, (float*)c->pc_blocks, pc_dev(c),
                           (const int*)eb.elems, sigma);
      }
    }
    FRX_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(KR_THREADS), 0, s, c->pc_isig, 1L, 1.0 / sigma);
  FRX_TRY(hipGetLastError());
  FRX_TRY(hipMemcpyAsync(c->ipin + 16, c->pc_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  FRX_TRY(hipStreamSynchronize(s));
  c->pc_built = c->ipin[16] == 0;
  c->pc_half = half;
  if (!c->pc_built) throw StatusErr{FR_E_NONPHYSICAL, "element-Jacobi preconditioner: a singular element block"};
}

// Iterations of the cycle just finished (read by gmres_run after its
// synchronisation) sizes the first graph of the next cycle.
void note_cycle(fr_ctx c, int mode, int prec_bytes, int iters) { c->cycle_iters[{mode, prec_bytes}] = iters; }

// Restarted GMRES on the device.  x (float64, device) receives the solution.
template <class TV>
fr_status gmres_run(fr_ctx c, const fr_gmres_opts& o, double* x, fr_gmres_stats* st, hipStream_t s,
                    double nF_known) {
  const long n = c->ndof;
  const int m = o.restart;
  GmresDev G = gdev(c);
  TV* V = (TV*)c->Vb;
  TV* w = (TV*)c->wv;
  TV* xv = (TV*)c->xv;
  // ||F|| (unless the caller has it), tolerance, budget
  // left preconditioning: the Krylov space of P^-1 A, the right-hand side
  // P^-1 F and the residual norms of the preconditioned system
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, c->ist + 5, o.precond);
  FRX_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, c->ist + 6, o.orthog == FR_ORTHO_CGS ? 1 : 0);
  FRX_TRY(hipGetLastError());
  if (o.precond) {
    FRX_TRY(hipMemcpyAsync(c->rb, c->Fb, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    pc_apply<double>(c, c->rb, nullptr, s);
  }
  const double nF = o.precond ? norm2(c, c->rb, s) : (nF_known >= 0.0 ? nF_known : norm2(c, c->Fb, s));
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(KR_THREADS), 0, s, x, n, 0.0);
  FRX_TRY(hipGetLastError());
  fr_gmres_stats stats{0, 0, 0.0, 1};
  if (nF == 0.0) {
    if (st) *st = stats;
    return FR_OK;
  }
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, c->sc + 1, nF);
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, c->sc + 2, o.tol);
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, c->ist + 2, 0);
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, c->ist + 3, o.max_iter);
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, c->ist + 4, m);
  FRX_TRY(hipGetLastError());
  double res = nF;
  int total = 0, cycles = 0;
  bool conv = false;
  while (true) {
    // restart residual r = F - A x (r = F at the start), preconditioned
    if (cycles == 0) {
      if (!o.precond) FRX_TRY(hipMemcpyAsync(c->rb, c->Fb, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    } else {
      hipLaunchKernelGGL((k_cast<double, TV>), dim3(grid_for(n)), dim3(KR_THREADS), 0, s, (const double*)x, xv, n);
      FRX_TRY(hipGetLastError());
      apply_A<TV>(c, o.jv_mode, xv, w, nullptr, s);
      hipLaunchKernelGGL((k_cast<TV, double>), dim3(grid_for(n)), dim3(KR_THREADS), 0, s, (const TV*)w, c->R1, n);
      FRX_TRY(hipGetLastError());
      lincomb(c, c->rb, 1.0, c->Fb, -1.0, c->R1, 0, nullptr, 0, nullptr, s);
      if (o.precond) pc_apply<double>(c, c->rb, nullptr, s);
    }
    dot_to<double>(c, c->rb, nullptr, c->sc + 9, nullptr, s);
    hipLaunchKernelGGL(k_cycle_start, dim3(1), dim3(1), 0, s, G, (const double*)(c->sc + 9));
    FRX_TRY(hipGetLastError());
    hipLaunchKernelGGL((k_scale<double, TV>), dim3(grid_for(n)), dim3(KR_THREADS), 0, s, (const double*)c->rb, V, n,
                       (const double*)(c->sc + 4), 0, (const int*)nullptr);
    FRX_TRY(hipGetLastError());
    arnoldi_cycle<TV>(c, o.jv_mode, m, o.use_graph != 0, s);
    hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(1), 0, s, G);
    FRX_TRY(hipGetLastError());
    hipLaunchKernelGGL((k_update_x<TV>), dim3(grid_for(n)), dim3(KR_THREADS), 0, s, (const TV*)V, n,
                       (const double*)G.y, (const int*)(c->ist + 1), x, n);
    FRX_TRY(hipGetLastError());
    FRX_TRY(hipMemcpyAsync(c->ipin, c->ist, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    FRX_TRY(hipMemcpyAsync(c->hpin, c->sc, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    FRX_TRY(hipStreamSynchronize(s));
    ++cycles;
    total = c->ipin[2];
    res = c->hpin[3];
    if (o.use_graph) note_cycle(c, o.jv_mode, (int)sizeof(TV), c->ipin[1]);
    if (res <= o.tol * nF) {
      conv = true;
      break;
    }
    if (total >= o.max_iter || c->ipin[1] == 0) break;
  }
  stats.iterations = total;
  stats.cycles = cycles;
  stats.rel_res = res / nF;
  stats.converged = conv ? 1 : 0;
  if (st) *st = stats;
  return conv ? FR_OK : FR_E_NOTCONVERGED;
}

// Prepare linearisation state and right-hand side, then run GMRES.
fr_status gmres_solve(fr_ctx c, const double* U, double shift, const double* F, double* dU, const fr_gmres_opts& o,
                      fr_gmres_stats* st, hipStream_t s, const double* R0_known, double nF_known = -1.0) {
  if (o.restart < 1 || o.max_iter < 1 || !(o.tol >= 0.0) || !(o.fd_eps >= 0.0) ||
      (o.jv_mode != FR_JV_EXACT && o.jv_mode != FR_JV_FD && o.jv_mode != FR_JV_FD_SCALED) ||
      (o.precision != FR_F64 && o.precision != FR_F32) || (o.orthog != FR_ORTHO_CGS2 && o.orthog != FR_ORTHO_CGS))
    throw StatusErr{FR_E_INVALID, "gmres options out of range"};
  if (o.orthog == FR_ORTHO_CGS && o.restart > 32)
    throw StatusErr{FR_E_INVALID, "one-pass Gram-Schmidt is built for restart <= 32"};
  if (o.precision == FR_F32 && o.jv_mode != FR_JV_EXACT)
    throw StatusErr{FR_E_UNSUPPORTED, "float32 GMRES needs the exact tangent"};
  if (o.restart > c->m_alloc)
    throw StatusErr{FR_E_INVALID, "restart " + std::to_string(o.restart) + " exceeds the reserved workspace (" +
                                      std::to_string(c->m_alloc) + "); call fr_reserve"};
  if (o.use_graph && !(c->graph_sets & graph_bit(o.jv_mode, o.precision)))
    throw StatusErr{FR_E_INVALID, "Arnoldi graphs of this mode and precision were not reserved (fr_reserve)"};
  if (o.precond < 0 || o.precond > 2) throw StatusErr{FR_E_INVALID, "gmres options out of range"};
  if (o.precond && (!c->pc_built || c->pc_prec != o.precision || c->pc_half != (o.precond == 2)))
    throw StatusErr{FR_E_INVALID, "no element-Jacobi preconditioner built in this precision and form (fr_precond_build)"};
  const long n = c->ndof;
  if (U != c->Ulin) FRX_TRY(hipMemcpyAsync(c->Ulin, U, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  if (F != c->Fb) FRX_TRY(hipMemcpyAsync(c->Fb, F, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, c->sc + 6, shift);
  hipLaunchKernelGGL((k_cast<double, float>), dim3(1), dim3(1), 0, s, (const double*)(c->sc + 6), c->sigf, 1L);
  FRX_TRY(hipGetLastError());
  if (o.jv_mode != FR_JV_EXACT) {
    // finite-difference step on the device: eps, or eps sqrt(1 + ||U||) (scaled)
    const double eps = o.fd_eps > 0 ? o.fd_eps : 1e-6;
    if (o.jv_mode == FR_JV_FD_SCALED) {
      dot_to<double>(c, c->Ulin, nullptr, c->sc + 12, nullptr, s);
      hipLaunchKernelGGL(k_fd_scaled_eps, dim3(1), dim3(1), 0, s, (const double*)(c->sc + 12), eps, c->sc + 7);
    } else {
      hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, c->sc + 7, eps);
    }
    FRX_TRY(hipGetLastError());
    if (R0_known) {
      FRX_TRY(hipMemcpyAsync(c->R0, R0_known, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    } else {
      ResCall<double> rc;
      rc.U = c->Ulin;
      rc.out = c->R0;
      FRX_TRY(launch_residual_f64(c->M, rc, s));
    }
  }
  if (o.precision == FR_F32) {
    hipLaunchKernelGGL((k_cast<double, float>), dim3(grid_for(n)), dim3(KR_THREADS), 0, s, (const double*)c->Ulin,
                       c->uf, n);
    FRX_TRY(hipGetLastError());
    return gmres_run<float>(c, o, dU, st, s, nF_known);
  }
  return gmres_run<double>(c, o, dU, st, s, nF_known);
}

// Tile tables of the fused launches: every degree bucket cut into blocks of
// 256 threads, all tiles of a stage sorted by decreasing work.  The items per
// tile (elements of one degree, or faces of one degree pair) are a shape of
// (scalar kind, stage, bucket code) that fr_autotune may change; the default
// fills the 256 threads within the stage's LDS cap.

// LDS bytes per item of a stage for the bucket code (n for elements, 8 nl + nh
// for interior faces)
size_t item_lds(bool ns, size_t sb, int st, int code) {
  if (st != 1) {
    const int n = code, n3 = n * n * n;
    const int tv = trace_lds_vals(ns, n, (int)sb);
    return st == 0 ? (size_t)tv * n3 * sb : (size_t)(5 * n3 + 30 * n * n) * sb;
  }
  const int nl = code / 8, nh = code % 8;
  return nl < nh ? (size_t)((ns ? 20 : 5) * nl * nl + 10 * nh * nh) * sb : 0;
}
// threads of one item: n^3 (elements) or nh^2 (faces)
int item_threads(int st, int code) { return st != 1 ? code * code * code : (code % 8) * (code % 8); }
// LDS cap per tile of a stage: the share of the blocks per CU it is built for
size_t stage_lds_cap(int sk, int st) { return std::min<size_t>(64 * 1024, 160 * 1024 / FRX_STAGE_WAVES[sk][st]); }
// the largest items per tile that fit 256 threads and the LDS cap
int max_items(bool ns, int sk, int st, int code) {
  const size_t per = item_lds(ns, scalar_bytes(sk), st, code);
  int k = std::max(1, FRX_MAX_THREADS / item_threads(st, code));
  while (k > 1 && per * k > stage_lds_cap(sk, st)) --k;
  return k;
}

// XCD-aware order of a tile table.  Workgroup b of a launch runs on XCD
// b mod 8 (the dispatcher deals workgroups to the XCDs round-robin), and each
// XCD has its own L2.  The heavy-first list is cut into runs of one bucket
// code; every run is split into 8 contiguous chunks, chunk x going to XCD x
// (the larger chunks to the XCDs with the fewest tiles so far), and the table
// interleaves the 8 sequences: entry 8 j + x is tile j of XCD x.  Each XCD so
// walks contiguous pieces of every bucket, heaviest first, and tiles whose
// face slots share cache lines meet in the same L2.  The sequences are padded
// to one length with empty tiles (code 0), which the kernels skip.
constexpr int N_XCD = 8;
std::vector<int4> xcd_order(const std::vector<int4>& t) {
  std::vector<std::vector<int4>> seq(N_XCD);
  size_t i = 0;
  while (i < t.size()) {
    size_t j = i;
    while (j < t.size() && t[j].x == t[i].x) ++j;
    const size_t m = j - i, q = m / N_XCD, r = m % N_XCD;
    std::vector<int> ord(N_XCD);
    for (int x = 0; x < N_XCD; ++x) ord[x] = x;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return seq[a].size() < seq[b].size(); });
    std::vector<size_t> len(N_XCD, q);
    for (size_t k = 0; k < r; ++k) ++len[ord[k]];
    size_t at = i;
    for (int x = 0; x < N_XCD; ++x) {
      seq[x].insert(seq[x].end(), t.begin() + at, t.begin() + at + len[x]);
      at += len[x];
    }
    i = j;
  }
  size_t L = 0;
  for (auto& v : seq) L = std::max(L, v.size());
  std::vector<int4> out(N_XCD * L, make_int4(0, 0, 0, 0));
  for (int x = 0; x < N_XCD; ++x)
    for (size_t k = 0; k < seq[x].size(); ++k) out[N_XCD * k + x] = seq[x][k];
  return out;
}

// The tile table of one stage of one scalar kind over element ranges er
// (n -> first, count) or face ranges fr (code, first, count, nl), with the
// chosen items per tile (c->shape; the defaults if use_shapes is false), in
// the XCD order; *lds receives the largest tile's LDS and *nint the length
// of the interior-face part.
std::vector<int4> make_tiles(fr_ctx c, int sk, int st, const std::map<int, std::pair<int, int>>& er,
                             const std::vector<std::tuple<int, int, int, int>>& fr, bool use_shapes, size_t* lds_out,
                             int* nint_out) {
  MeshDev& M = c->M;
  const bool ns = M.physics == FR_NAVIER_STOKES;
  std::vector<std::pair<double, int4>> tiles;
  size_t lds = 0;
  auto items = [&](int code) {
    if (!use_shapes) return max_items(ns, sk, st, code);
    auto it = c->shape[sk][st].find(code);
    return it != c->shape[sk][st].end() ? it->second : max_items(ns, sk, st, code);
  };
  if (st != 1) {
    for (auto& kv : er) {
      const int n = kv.first, first = kv.second.first, count = kv.second.second;
      const int epb = items(n);
      lds = std::max(lds, epb * item_lds(ns, scalar_bytes(sk), st, n));
      for (int i = 0; i < count; i += epb) {
        const int cnt = std::min(epb, count - i);
        tiles.push_back({(double)cnt * n * n * n * n, make_int4(n, first + i, cnt, epb)});
      }
    }
  } else {
    for (auto& f : fr) {
      const int code = std::get<0>(f), first = std::get<1>(f), count = std::get<2>(f);
      if (code >= 64) {
        const int n = code - 64, per = std::max(1, 256 / (n * n));
        for (int i = 0; i < count; i += per)
          tiles.push_back({(double)std::min(per, count - i) * n * n * 2.0,
                           make_int4(code, first + i, std::min(per, count - i), per)});
      } else {
        const int nl = code / 8, nh = code % 8;
        const int fpb = items(code);
        lds = std::max(lds, fpb * item_lds(ns, scalar_bytes(sk), st, code));
        for (int i = 0; i < count; i += fpb)
          tiles.push_back({(double)std::min(fpb, count - i) * nh * nh * (nl < nh ? 1.5 : 1.0),
                           make_int4(code, first + i, std::min(fpb, count - i), fpb)});
      }
    }
  }
  // by decreasing work; in the face stage interior-face tiles (code < 64)
  // before boundary-face tiles, so that the two-pass face stage can launch
  // each group on its own
  std::stable_sort(tiles.begin(), tiles.end(), [](const std::pair<double, int4>& x, const std::pair<double, int4>& y) {
    const bool bx = x.second.x >= 64, by = y.second.x >= 64;
    if (bx != by) return !bx;
    return x.first > y.first;
  });
  std::vector<int4> t_int, t_bnd;
  for (auto& x : tiles) (x.second.x < 64 ? t_int : t_bnd).push_back(x.second);
  std::vector<int4> t = xcd_order(t_int);
  *nint_out = (int)t.size();
  if (!t_bnd.empty()) {
    const std::vector<int4> tb = xcd_order(t_bnd);
    t.insert(t.end(), tb.begin(), tb.end());
  }
  *lds_out = lds;
  return t;
}

// (Re)builds the tile table of one stage of one scalar kind from the chosen
// items per tile (c->shape), into the table allocated for the worst case.
void plan_stage(fr_ctx c, int sk, int st) {
  FusedPlan& P = c->M.plan[sk];
  size_t lds = 0;
  int nint = 0;
  const std::vector<int4> t = make_tiles(c, sk, st, c->erange, c->frange, true, &lds, &nint);
  if ((int)t.size() > c->plan_cap[st]) throw StatusErr{FR_E_INVALID, "tile table larger than its allocation"};
  if (st == 1) P.n_interior = nint;
  P.count[st] = (int)t.size();
  P.lds[st] = lds;
  if (!t.empty()) FRX_TRY(hipMemcpy(P.tiles[st], t.data(), sizeof(int4) * t.size(), hipMemcpyHostToDevice));
}

void build_fused_plans(fr_ctx c, const fr_mesh_desc* d, const std::map<std::pair<int, int>, std::vector<int4>>& fmap,
                       const std::map<int, std::vector<int4>>& bmap) {
  MeshDev& M = c->M;
  const int E = d->n_elem;
  std::vector<int> all;
  std::map<int, std::pair<int, int>>& erange = c->erange;  // n -> (first, count)
  for (int n = NMAX; n >= 2; --n) {
    const int first = (int)all.size();
    for (int e = 0; e < E; ++e)
      if (d->elem_p[e] + 1 == n) all.push_back(e);
    if ((int)all.size() > first) erange[n] = {first, (int)all.size() - first};
  }
  std::vector<int4> faces;
  std::vector<std::tuple<int, int, int, int>>& frange = c->frange;  // (code, first, count, nl)
  for (auto it = fmap.rbegin(); it != fmap.rend(); ++it) {
    frange.emplace_back(8 * it->first.first + it->first.second, (int)faces.size(), (int)it->second.size(), it->first.first);
    faces.insert(faces.end(), it->second.begin(), it->second.end());
  }
  for (auto it = bmap.rbegin(); it != bmap.rend(); ++it) {
    frange.emplace_back(64 + it->first, (int)faces.size(), (int)it->second.size(), it->first);
    faces.insert(faces.end(), it->second.begin(), it->second.end());
  }
  M.all_ids = (int*)c->dalloc(sizeof(int) * std::max<size_t>(1, all.size()));
  FRX_TRY(hipMemcpy(M.all_ids, all.data(), sizeof(int) * all.size(), hipMemcpyHostToDevice));
  std::vector<int4> all_recs;
  for (int e : all) all_recs.push_back(make_int4(e, (int)c->sp_off_h[e], c->fp_off_h[e], 0));
  M.all_elems = (int4*)c->dalloc(sizeof(int4) * std::max<size_t>(1, all_recs.size()));
  FRX_TRY(hipMemcpy(M.all_elems, all_recs.data(), sizeof(int4) * all_recs.size(), hipMemcpyHostToDevice));
  c->faces_h = faces;
  M.all_faces = (int4*)c->dalloc(sizeof(int4) * std::max<size_t>(1, faces.size()));
  if (!faces.empty())
    FRX_TRY(hipMemcpy(M.all_faces, faces.data(), sizeof(int4) * faces.size(), hipMemcpyHostToDevice));
  const bool ns = d->physics == FR_NAVIER_STOKES;
  // tile tables sized for one item per tile, so that any shape fits
  // (plus the padding of the XCD order: under 8 per run of one bucket code)
  const int pad = N_XCD * (2 * (int)(erange.size() + frange.size()) + 2);
  c->plan_cap[0] = c->plan_cap[2] = std::max(1, E) + pad;
  c->plan_cap[1] = std::max<int>(1, (int)faces.size()) + pad;
  for (int sk = 0; sk < SK_COUNT; ++sk)
    for (int st = 0; st < 3; ++st) {
      M.plan[sk].tiles[st] = (int4*)c->dalloc(sizeof(int4) * c->plan_cap[st]);
      plan_stage(c, sk, st);
    }
  const size_t cap = 64 * 1024;
  // adjoint (float64): LDS per element 5 n^3 (trace_rev) and 5 n^3 + 30 n^2
  // (div_rev); per mixed face (NV + 10) nl^2 + NV nh^2
  FusedPlan& V = M.vplan;
  for (int st = 0; st < 3; ++st) {
    std::vector<std::pair<double, int4>> tiles;
    size_t lds = 0;
    if (st != 1) {
      for (auto& kv : erange) {
        const int n = kv.first, n3 = n * n * n;
        const size_t per_el = (size_t)(5 * n3 + (st == 2 ? 30 * n * n : 0)) * 8;
        int epb = std::max(1, 256 / n3);
        while (epb > 1 && epb * per_el > cap) --epb;
        lds = std::max(lds, epb * per_el);
        for (int i = 0; i < kv.second.second; i += epb) {
          const int cnt = std::min(epb, kv.second.second - i);
          tiles.push_back({(double)cnt * n3 * n, make_int4(n, kv.second.first + i, cnt, epb)});
        }
      }
    } else {
      const int nv = ns ? 20 : 5;
      for (auto& fr : frange) {
        const int code = std::get<0>(fr), first = std::get<1>(fr), count = std::get<2>(fr);
        if (code >= 64) {
          const int n = code - 64, per = std::max(1, 256 / (n * n));
          for (int i = 0; i < count; i += per)
            tiles.push_back({(double)std::min(per, count - i) * n * n * 2.0,
                             make_int4(code, first + i, std::min(per, count - i), per)});
        } else {
          const int nl = code / 8, nh = code % 8;
          const size_t per_face = nl < nh ? (size_t)((nv + 10) * nl * nl + nv * nh * nh) * 8 : 0;
          int fpb = std::max(1, 256 / (nh * nh));
          while (fpb > 1 && fpb * per_face > cap) --fpb;
          lds = std::max(lds, fpb * per_face);
          for (int i = 0; i < count; i += fpb)
            tiles.push_back({(double)std::min(fpb, count - i) * nh * nh * (nl < nh ? 1.5 : 1.0),
                             make_int4(code, first + i, std::min(fpb, count - i), fpb)});
        }
      }
    }
    // by decreasing work, interior-face tiles before boundary-face tiles
    std::stable_sort(tiles.begin(), tiles.end(), [](const std::pair<double, int4>& x, const std::pair<double, int4>& y) {
      const bool bx = x.second.x >= 64, by = y.second.x >= 64;
      if (bx != by) return !bx;
      return x.first > y.first;
    });
    std::vector<int4> t_int, t_bnd;
    for (auto& x : tiles) (x.second.x < 64 ? t_int : t_bnd).push_back(x.second);
    std::vector<int4> t = xcd_order(t_int);
    if (st == 1) V.n_interior = (int)t.size();
    if (!t_bnd.empty()) {
      const std::vector<int4> tb = xcd_order(t_bnd);
      t.insert(t.end(), tb.begin(), tb.end());
    }
    V.count[st] = (int)t.size();
    V.lds[st] = lds;
    V.tiles[st] = (int4*)c->dalloc(sizeof(int4) * std::max<size_t>(1, t.size()));
    if (!t.empty()) FRX_TRY(hipMemcpy(V.tiles[st], t.data(), sizeof(int4) * t.size(), hipMemcpyHostToDevice));
  }
}

// The fused subsets of the preconditioner assembly (see pc_sub): per colour
// k and size n, the elements of colour k with n_e >= n by degree bucket, the
// interior faces with a side among them and their boundary faces, both in
// the order of the full face list, and the tiles of the three stages of
// every scalar kind with the default items per tile.  Built once, by
// fr_reserve with preconditioner storage.
void build_pc_subsets(fr_ctx c) {
  const int E = c->M.E;
  const std::vector<int>& colour = c->pc_colour;
  for (size_t k = 0; k < c->pc_sub.size(); ++k)
    for (int nmin = 2; nmin <= NMAX; ++nmin) {
      if (c->pc_sub[k][nmin]) continue;
      auto in = [&](int e) { return colour[e] == (int)k && c->p[e] + 1 >= nmin; };
      std::vector<int4> recs;
      std::map<int, std::pair<int, int>> er;
      for (int n = NMAX; n >= nmin; --n) {
        const int first = (int)recs.size();
        for (int e = 0; e < E; ++e)
          if (colour[e] == (int)k && c->p[e] + 1 == n)
            recs.push_back(make_int4(e, (int)c->sp_off_h[e], c->fp_off_h[e], 0));
        if ((int)recs.size() > first) er[n] = {first, (int)recs.size() - first};
      }
      if (recs.empty()) continue;
      std::vector<int4> faces;
      std::vector<std::tuple<int, int, int, int>> fr;
      for (auto& f : c->frange) {
        const int code = std::get<0>(f), first0 = std::get<1>(f), count0 = std::get<2>(f);
        const int first = (int)faces.size();
        for (int i = first0; i < first0 + count0; ++i) {
          const int4 F = c->faces_h[i];
          // interior record (L, R, ...), boundary record (e, f, bc, slot)
          if (in(F.x) || (code < 64 && in(F.y))) faces.push_back(F);
        }
        if ((int)faces.size() > first) fr.emplace_back(code, first, (int)faces.size() - first, std::get<3>(f));
      }
      auto S = std::make_unique<FusedSubset>();
      int4* de = (int4*)c->dalloc(sizeof(int4) * recs.size());
      FRX_TRY(hipMemcpy(de, recs.data(), sizeof(int4) * recs.size(), hipMemcpyHostToDevice));
      S->elems = de;
      int4* df = (int4*)c->dalloc(sizeof(int4) * std::max<size_t>(1, faces.size()));
      if (!faces.empty()) FRX_TRY(hipMemcpy(df, faces.data(), sizeof(int4) * faces.size(), hipMemcpyHostToDevice));
      S->faces = df;
      for (int sk = 0; sk < SK_COUNT; ++sk)
        for (int st = 0; st < 3; ++st) {
          size_t lds = 0;
          int nint = 0;
          const std::vector<int4> t = make_tiles(c, sk, st, er, fr, false, &lds, &nint);
          FusedPlan& P = S->plan[sk];
          if (st == 1) P.n_interior = nint;
          P.count[st] = (int)t.size();
          P.lds[st] = lds;
          P.tiles[st] = (int4*)c->dalloc(sizeof(int4) * std::max<size_t>(1, t.size()));
          if (!t.empty()) FRX_TRY(hipMemcpy(P.tiles[st], t.data(), sizeof(int4) * t.size(), hipMemcpyHostToDevice));
        }
      c->pc_sub[k][nmin] = std::move(S);
    }
}

void validate_desc(const fr_mesh_desc* d) {
  if (!d) throw StatusErr{FR_E_INVALID, "null descriptor"};
  if (d->n_elem <= 0 || !d->elem_xyz || !d->elem_nbr || !d->elem_p)
    throw StatusErr{FR_E_INVALID, "empty mesh or null arrays"};
  if (d->physics != FR_EULER && d->physics != FR_NAVIER_STOKES) throw StatusErr{FR_E_INVALID, "physics"};
  if (d->flux != FR_ROE && d->flux != FR_RUSANOV) throw StatusErr{FR_E_INVALID, "flux"};
  if (!(d->gamma > 1.0) || !(d->mu >= 0.0) || !(d->prandtl > 0.0)) throw StatusErr{FR_E_INVALID, "gas constants"};
  const int E = d->n_elem;
  for (int e = 0; e < E; ++e) {
    if (d->elem_p[e] < 1 || d->elem_p[e] > 5) throw StatusErr{FR_E_INVALID, "degree outside 1..5 at element " + std::to_string(e)};
    for (int f = 0; f < 6; ++f) {
      const int nb = d->elem_nbr[6 * e + f];
      if (nb >= E || (nb < 0 && nb != FR_BC_WALL && nb != FR_BC_FARFIELD))
        throw StatusErr{FR_E_INVALID, "neighbour id out of range at element " + std::to_string(e)};
      if (nb >= 0 && d->elem_nbr[6 * nb + (f ^ 1)] != e)
        throw StatusErr{FR_E_INVALID, "neighbour relation not symmetric at element " + std::to_string(e)};
      if (nb >= 0 && (f & 1)) {
        // L's +d face vertices must match R's -d face vertices up to one translation
        const int dd = f >> 1;
        const double* XL = d->elem_xyz + 24L * e;
        const double* XR = d->elem_xyz + 24L * nb;
        double t[3] = {0, 0, 0}, h = 0.0;
        for (int c = 0; c < 3; ++c) h = std::max(h, std::fabs(XL[3 * 7 + c] - XL[c]));
        bool first = true;
        for (int v = 0; v < 8; ++v) {
          if (!((v >> dd) & 1)) continue;
          const int vr = v & ~(1 << dd);
          for (int c = 0; c < 3; ++c) {
            const double dv = XR[3 * vr + c] - XL[3 * v + c];
            if (first) t[c] = dv;
            else if (std::fabs(dv - t[c]) > 1e-9 * std::max(1.0, h))
              throw StatusErr{FR_E_INVALID, "non-conforming face between elements " + std::to_string(e) + " and " +
                                                std::to_string(nb)};
          }
          first = false;
        }
      }
    }
  }
}

}  // namespace

// ======================================================================= C ABI
extern "C" {

fr_status fr_create(const fr_mesh_desc* d, fr_ctx* out) {
  if (!out) return fail(nullptr, FR_E_INVALID, "null output handle");
  *out = nullptr;
  fr_ctx c = nullptr;
  fr_status st = guarded(nullptr, [&]() -> fr_status {
    validate_desc(d);
    std::unique_ptr<fr_ctx_s> C(new fr_ctx_s);
    FRX_TRY(hipGetDevice(&C->dev));
    C->scratch_dev = scratch_on_device(C->dev);
    ensure_tables(C->dev);
    MeshDev& M = C->M;
    const int E = d->n_elem;
    M.E = E;
    M.physics = d->physics;
    M.flux = d->flux;
    C->p.assign(d->elem_p, d->elem_p + E);
    std::vector<int> sp(E), fp(E);
    C->sp_off_h.resize(E + 1);
    long nsp = 0, nfp = 0;
    for (int e = 0; e < E; ++e) {
      const int n = d->elem_p[e] + 1;
      sp[e] = (int)nsp;
      C->sp_off_h[e] = nsp;
      nsp += (long)n * n * n;
    }
    // face slots (internal) in the order of the fused element list: degree
    // buckets from the highest, mesh order inside a bucket, so that the
    // elements of a tile, and consecutive tiles, own contiguous slots
    for (int n = NMAX; n >= 2; --n)
      for (int e = 0; e < E; ++e)
        if (d->elem_p[e] + 1 == n) {
          fp[e] = (int)nfp;
          nfp += 6L * n * n;
        }
    C->sp_off_h[E] = nsp;
    C->fp_off_h = fp;
    // (30 nfp < 2^31 also keeps face-slot offsets below 2^28, as the packed
    // interior-face records need)
    if (5 * nsp >= (1L << 31) || 30 * nfp >= (1L << 31)) throw StatusErr{FR_E_INVALID, "mesh too large for 32-bit indices"};
    M.nsp = (int)nsp;
    M.nfp = (int)nfp;
    C->ndof = 5 * nsp;
    // trilinear monomial coefficients
    std::vector<double> geo(24L * E);
    std::vector<float> geof(24L * E);
    for (int e = 0; e < E; ++e) {
      const double* X = d->elem_xyz + 24L * e;
      for (int mnm = 0; mnm < 8; ++mnm) {
        // monomials: 1, r0, r1, r2, r0 r1, r1 r2, r0 r2, r0 r1 r2
        static const int use[8][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {0, 1, 1}, {1, 0, 1}, {1, 1, 1}};
        for (int c = 0; c < 3; ++c) {
          double s = 0.0;
          for (int v = 0; v < 8; ++v) {
            double f = 0.125;
            for (int i = 0; i < 3; ++i)
              if (use[mnm][i]) f *= ((v >> i) & 1) ? 1.0 : -1.0;
            s += f * X[3 * v + c];
          }
          geo[24L * e + 3 * mnm + c] = s;
          geof[24L * e + 3 * mnm + c] = (float)s;
        }
      }
    }
    M.sp_off = (int*)C->dalloc(sizeof(int) * E);
    M.fp_off = (int*)C->dalloc(sizeof(int) * E);
    M.geo_d = (double*)C->dalloc(sizeof(double) * 24L * E);
    M.geo_f = (float*)C->dalloc(sizeof(float) * 24L * E);
    FRX_TRY(hipMemcpy(M.sp_off, sp.data(), sizeof(int) * E, hipMemcpyHostToDevice));
    FRX_TRY(hipMemcpy(M.fp_off, fp.data(), sizeof(int) * E, hipMemcpyHostToDevice));
    FRX_TRY(hipMemcpy(M.geo_d, geo.data(), sizeof(double) * 24L * E, hipMemcpyHostToDevice));
    FRX_TRY(hipMemcpy(M.geo_f, geof.data(), sizeof(float) * 24L * E, hipMemcpyHostToDevice));
    // degree buckets
    for (int n = 2; n <= NMAX; ++n) {
      std::vector<int> ids;
      for (int e = 0; e < E; ++e)
        if (d->elem_p[e] + 1 == n) ids.push_back(e);
      if (ids.empty()) continue;
      ElemBucket b;
      b.n = n;
      b.count = (int)ids.size();
      b.elems = (int*)C->dalloc(sizeof(int) * ids.size());
      FRX_TRY(hipMemcpy(b.elems, ids.data(), sizeof(int) * ids.size(), hipMemcpyHostToDevice));
      std::vector<int4> recs;
      for (int e : ids) recs.push_back(make_int4(e, sp[e], fp[e], 0));
      b.recs = (int4*)C->dalloc(sizeof(int4) * recs.size());
      FRX_TRY(hipMemcpy(b.recs, recs.data(), sizeof(int4) * recs.size(), hipMemcpyHostToDevice));
      M.eb.push_back(b);
    }
    // face buckets by (n_low, n_high); boundary faces by n
    std::map<std::pair<int, int>, std::vector<int4>> fmap;
    std::map<int, std::vector<int4>> bmap;
    for (int e = 0; e < E; ++e)
      for (int f = 0; f < 6; ++f) {
        const int nb = d->elem_nbr[6 * e + f];
        const int ne = d->elem_p[e] + 1;
        if (nb >= 0) {
          if (!(f & 1)) continue;
          const int nr = d->elem_p[nb] + 1;
          // (L, R, first slot of L's +d face, first slot of R's -d face | d << 28 | low_is_R << 30)
          const int oL = fp[e] + f * ne * ne, oR = fp[nb] + (f - 1) * nr * nr;
          fmap[{std::min(ne, nr), std::max(ne, nr)}].push_back(
              make_int4(e, nb, oL, oR | ((f >> 1) << 28) | ((nr < ne ? 1 : 0) << 30)));
        } else {
          bmap[ne].push_back(make_int4(e, f, nb, fp[e] + f * ne * ne));
        }
      }
    for (auto& kv : fmap) {
      FaceBucket b;
      b.nl = kv.first.first;
      b.nh = kv.first.second;
      b.count = (int)kv.second.size();
      b.faces = (int4*)C->dalloc(sizeof(int4) * kv.second.size());
      FRX_TRY(hipMemcpy(b.faces, kv.second.data(), sizeof(int4) * kv.second.size(), hipMemcpyHostToDevice));
      M.fb.push_back(b);
    }
    for (auto& kv : bmap) {
      BFaceBucket b;
      b.n = kv.first;
      b.count = (int)kv.second.size();
      b.faces = (int4*)C->dalloc(sizeof(int4) * kv.second.size());
      FRX_TRY(hipMemcpy(b.faces, kv.second.data(), sizeof(int4) * kv.second.size(), hipMemcpyHostToDevice));
      M.bb.push_back(b);
    }
    for (int sk = 0; sk < SK_COUNT; ++sk) default_shapes(M, sk);
    build_fused_plans(C.get(), d, fmap, bmap);
    // preconditioner records and a colouring of the elements in which no two
    // face neighbours share a colour (greedy, in mesh order)
    {
      std::vector<int> colour(E, -1);
      int ncol = 0;
      for (int e = 0; e < E; ++e) {
        unsigned used = 0;
        for (int f = 0; f < 6; ++f) {
          const int nb = d->elem_nbr[6 * e + f];
          if (nb >= 0 && colour[nb] >= 0) used |= 1u << colour[nb];
        }
        int k = 0;
        while (used & (1u << k)) ++k;
        colour[e] = k;
        ncol = std::max(ncol, k + 1);
      }
      std::vector<int4> recs(E);
      std::vector<long> boff(E);
      std::vector<int> poff(E);
      long b = 0;
      int pv = 0;
      for (int e = 0; e < E; ++e) {
        const int n = d->elem_p[e] + 1, N = 5 * n * n * n;
        recs[e] = make_int4(e, sp[e], n, 0);
        boff[e] = b;
        poff[e] = pv;
        b += pc_block_size(N);
        pv += N;
        C->pc_nmax = std::max(C->pc_nmax, N);
      }
      C->pc_recs = (int4*)C->dalloc(sizeof(int4) * E);
      C->pc_boff = (long*)C->dalloc(sizeof(long) * E);
      C->pc_poff = (int*)C->dalloc(sizeof(int) * E);
      C->pc_piv = (int*)C->dalloc(sizeof(int) * std::max(1, pv));
      C->pc_flag = (int*)C->dalloc(sizeof(int) * 4);
      C->pc_isig = (double*)C->dalloc(sizeof(double) * 2);
      FRX_TRY(hipMemcpy(C->pc_recs, recs.data(), sizeof(int4) * E, hipMemcpyHostToDevice));
      FRX_TRY(hipMemcpy(C->pc_boff, boff.data(), sizeof(long) * E, hipMemcpyHostToDevice));
      FRX_TRY(hipMemcpy(C->pc_poff, poff.data(), sizeof(int) * E, hipMemcpyHostToDevice));
      for (int k = 0; k < ncol; ++k) {
        std::vector<int4> cr;
        std::vector<int> ci;
        for (int e = 0; e < E; ++e)
          if (colour[e] == k) {
            cr.push_back(recs[e]);
            ci.push_back(e);
          }
        int4* crd = (int4*)C->dalloc(sizeof(int4) * std::max<size_t>(1, cr.size()));
        int* cid = (int*)C->dalloc(sizeof(int) * std::max<size_t>(1, ci.size()));
        FRX_TRY(hipMemcpy(crd, cr.data(), sizeof(int4) * cr.size(), hipMemcpyHostToDevice));
        FRX_TRY(hipMemcpy(cid, ci.data(), sizeof(int) * ci.size(), hipMemcpyHostToDevice));
        C->pc_crecs.push_back(crd);
        C->pc_cidx.push_back(cid);
        C->pc_ccount.push_back((int)cr.size());
      }
      C->pc_colour = colour;
      C->pc_sub.resize(ncol);
    }
    // gas
    const double kappa = d->mu * d->gamma / ((d->gamma - 1.0) * d->prandtl);
    M.gas_d.gamma = d->gamma;
    M.gas_d.gm1 = d->gamma - 1.0;
    M.gas_d.mu = d->mu;
    M.gas_d.kappa = kappa;
    M.gas_f.gamma = (float)d->gamma;
    M.gas_f.gm1 = (float)(d->gamma - 1.0);
    M.gas_f.mu = (float)d->mu;
    M.gas_f.kappa = (float)kappa;
    for (int v = 0; v < 5; ++v) {
      M.gas_d.ff[v] = d->farfield[v];
      M.gas_f.ff[v] = (float)d->farfield[v];
    }
    M.facebuf = C->dalloc(30L * nfp * 16);
    M.fgeo_d = (double*)C->dalloc(sizeof(double) * 5L * nfp);
    M.fgeo_f = (float*)C->dalloc(sizeof(float) * 5L * nfp);
    FRX_TRY(launch_face_geometry(M, nullptr));
    M.p_dev = (int8_t*)C->dalloc(E);
    FRX_TRY(hipMemcpy(M.p_dev, d->elem_p, E, hipMemcpyHostToDevice));
    M.nbr = (int*)C->dalloc(sizeof(int) * 6L * E);
    FRX_TRY(hipMemcpy(M.nbr, d->elem_nbr, sizeof(int) * 6L * E, hipMemcpyHostToDevice));
    M.eta_w = (double*)C->dalloc(sizeof(double) * (E + 8));
    M.psel = (int8_t*)C->dalloc(2L * E);
    M.flag = (int*)C->dalloc(sizeof(int) * 4);
    FRX_TRY(hipMemset(M.flag, 0, sizeof(int) * 4));
    C->t0 = (double*)C->dalloc(sizeof(double) * C->ndof);
    C->t1 = (double*)C->dalloc(sizeof(double) * C->ndof);
    C->t2 = (double*)C->dalloc(sizeof(double) * C->ndof);
    C->uf = (float*)C->dalloc(sizeof(float) * C->ndof);
    C->hpin = (double*)host_take();
    C->ipin = (int*)host_take();
    ensure_krylov(C.get(), 1);
    FRX_TRY(hipDeviceSynchronize());
    c = C.release();
    return FR_OK;
  });
  if (st == FR_OK) *out = c;
  return st;
}

fr_status fr_trim(void) {
  BlockCache& C = block_cache();
  std::lock_guard<std::mutex> lock(C.mu);
  for (auto& dv : C.dev_free) {
    for (auto& kv : dv.second) (void)hipFree(kv.second);
    dv.second.clear();
  }
  for (auto& kv : C.dev_bytes) kv.second = 0;
  for (void* p : C.host_free) (void)hipHostFree(p);
  C.host_free.clear();
  return FR_OK;
}

fr_status fr_destroy(fr_ctx c) {
  if (!c) return FR_E_INVALID;
  (void)hipDeviceSynchronize();
  delete c;
  return FR_OK;
}

fr_status fr_layout(fr_ctx c, int64_t* n_dof, int64_t* sp_offset) {
  if (!c) return FR_E_INVALID;
  if (n_dof) *n_dof = c->ndof;
  if (sp_offset) std::copy(c->sp_off_h.begin(), c->sp_off_h.end(), sp_offset);
  return FR_OK;
}

fr_status fr_reserve(fr_ctx c, int32_t max_restart, int32_t graph_sets) {
  if (!c) return FR_E_INVALID;
  const int gbits = FR_GRAPHS_F64_EXACT | FR_GRAPHS_F32_EXACT | FR_GRAPHS_F64_FD | FR_GRAPHS_F64_FD_SCALED;
  const int pbits = FR_RESERVE_PRECOND_F64 | FR_RESERVE_PRECOND_F32;
  if (max_restart < 1 || max_restart > 200 || (graph_sets & ~(gbits | pbits)) || (graph_sets & pbits) == pbits)
    return fail(c, FR_E_INVALID, "fr_reserve: max_restart outside 1..200, unknown bits or two preconditioner precisions");
  return guarded(c, [&]() -> fr_status {
    FRX_TRY(hipDeviceSynchronize());
    ensure_krylov(c, max_restart);
    if (!c->es) c->es = (double*)c->dalloc(sizeof(double) * 11 * c->ndof);
    const int want = (graph_sets & FR_RESERVE_PRECOND_F64) ? FR_F64 : ((graph_sets & FR_RESERVE_PRECOND_F32) ? FR_F32 : -1);
    if (want >= 0 && want != c->pc_prec) {
      // one block of N_e^2 entries per element, N_e = 5 (p_e + 1)^3
      if (c->pc_blocks) c->dfree(c->pc_blocks);
      long entries = 0;
      for (int e = 0; e < c->M.E; ++e) entries += pc_block_size(5 * (c->p[e] + 1) * (c->p[e] + 1) * (c->p[e] + 1));
      c->pc_blocks = c->dalloc((size_t)entries * (want == FR_F64 ? sizeof(double) : sizeof(float)));
      c->pc_prec = want;
      c->pc_built = false;
    }
    if (want >= 0) build_pc_subsets(c);
    c->graph_sets |= (graph_sets & gbits);
    instantiate_graphs(c);
    FRX_TRY(hipDeviceSynchronize());
    return FR_OK;
  });
}

// true if the byte ranges [a, a + na) and [b, b + nb) share memory
bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + nb && y < x + na;
}

fr_status fr_residual(fr_ctx c, const double* U, double* R, void* stream) {
  if (!c) return FR_E_INVALID;
  const size_t nb = sizeof(double) * c->ndof;
  if (!U || !R || overlap(U, nb, R, nb)) return fail(c, FR_E_INVALID, "fr_residual: bad arguments");
  return guarded(c, [&]() -> fr_status {
    ResCall<double> rc;
    rc.U = U;
    rc.out = R;
    FRX_TRY(launch_residual_f64(c->M, rc, S(stream)));
    return FR_OK;
  });
}

fr_status fr_residual_noalloc(fr_ctx c, const double* U, double* R, void* stream) {
  if (!c) return FR_E_INVALID;
  const size_t nb = sizeof(double) * c->ndof;
  if (!U || !R || overlap(U, nb, R, nb)) return fail(c, FR_E_INVALID, "fr_residual_noalloc: bad arguments");
  // the float64 stages keep 30 face-slot values per own face point (q, grad q,
  // q_com - q, f_com . S)
  const size_t need = 30 * sizeof(double) * (size_t)c->M.nfp;
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(c, FR_E_INVALID, "fr_residual_noalloc: the mesh needs " + std::to_string(need) +
                                     " bytes of face-slot scratch, more than the " +
                                     std::to_string(NOALLOC_SCRATCH_BYTES) + " it holds (use fr_residual)");
  return guarded(c, [&]() -> fr_status {
    int dev = -1;
    FRX_TRY(hipGetDevice(&dev));
    if (dev != c->dev) throw StatusErr{FR_E_INVALID, "fr_residual_noalloc: the context's device is not current"};
    // the same kernels as fr_residual, with the face slots in the static scratch
    struct Swap {
      MeshDev& M;
      void* saved;
      ~Swap() { M.facebuf = saved; }
    } swap{c->M, c->M.facebuf};
    c->M.facebuf = c->scratch_dev;
    ResCall<double> rc;
    rc.U = U;
    rc.out = R;
    FRX_TRY(launch_residual_f64(c->M, rc, S(stream)));
    return FR_OK;
  });
}

fr_status fr_residual_jvp(fr_ctx c, const double* U, const double* v, double* R, double* Jv, void* stream) {
  if (!c) return FR_E_INVALID;
  const size_t nb = sizeof(double) * c->ndof;
  if (!U || !v || !R || !Jv || overlap(R, nb, U, nb) || overlap(Jv, nb, v, nb) || overlap(R, nb, Jv, nb) ||
      overlap(R, nb, v, nb) || overlap(Jv, nb, U, nb))
    return fail(c, FR_E_INVALID, "fr_residual_jvp: bad arguments");
  return guarded(c, [&]() -> fr_status {
    ResCall<double> rc;
    rc.U = U;
    rc.V = v;
    rc.out = Jv;
    rc.out_val = R;
    FRX_TRY(launch_residual_dual64(c->M, rc, S(stream)));
    return FR_OK;
  });
}

fr_status fr_jvp(fr_ctx c, const double* U, const void* v, void* Jv, int32_t prec, int32_t mode, double eps,
                 void* stream) {
  if (!c) return FR_E_INVALID;
  const size_t nb = sizeof(double) * c->ndof, nv = (prec == FR_F32 ? sizeof(float) : sizeof(double)) * c->ndof;
  if (!U || !v || !Jv || overlap(v, nv, Jv, nv) || overlap(U, nb, Jv, nv))
    return fail(c, FR_E_INVALID, "fr_jvp: bad arguments");
  if (prec != FR_F64 && prec != FR_F32) return fail(c, FR_E_INVALID, "fr_jvp: precision");
  if (mode != FR_JV_EXACT && mode != FR_JV_FD && mode != FR_JV_FD_SCALED) return fail(c, FR_E_INVALID, "fr_jvp: mode");
  if (mode != FR_JV_EXACT && prec != FR_F64) return fail(c, FR_E_UNSUPPORTED, "fr_jvp: finite differences need float64");
  if (!(eps >= 0.0)) return fail(c, FR_E_INVALID, "fr_jvp: fd_eps must be >= 0 (0: the default 1e-6)");
  return guarded(c, [&]() -> fr_status {
    hipStream_t s = S(stream);
    const long n = c->ndof;
    if (mode == FR_JV_EXACT && prec == FR_F64) {
      ResCall<double> rc;
      rc.U = U;
      rc.V = (const double*)v;
      rc.out = (double*)Jv;
      FRX_TRY(launch_residual_dual64(c->M, rc, s));
    } else if (mode == FR_JV_EXACT) {
      hipLaunchKernelGGL((k_cast<double, float>), dim3(grid_for(n)), dim3(KR_THREADS), 0, s, U, c->uf, n);
      FRX_TRY(hipGetLastError());
      ResCall<float> rc;
      rc.U = c->uf;
      rc.V = (const float*)v;
      rc.out = (float*)Jv;
      FRX_TRY(launch_residual_dual32(c->M, rc, s));
    } else {
      const double e = eps > 0 ? eps : 1e-6;
      double* nrm = c->sc + 10;
      double* epsd = c->sc + 13;
      dot_to<double>(c, (const double*)v, nullptr, nrm, nullptr, s);
      if (mode == FR_JV_FD_SCALED) {
        dot_to<double>(c, U, nullptr, c->sc + 14, nullptr, s);
        hipLaunchKernelGGL(k_fd_scaled_eps, dim3(1), dim3(1), 0, s, (const double*)(c->sc + 14), e, epsd);
      } else {
        hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, epsd, e);
      }
      hipLaunchKernelGGL((k_fd_perturb<double>), dim3(grid_for(n)), dim3(KR_THREADS), 0, s, U, (const double*)v, nrm,
                         (const double*)epsd, c->t0, n, (const int*)nullptr);
      FRX_TRY(hipGetLastError());
      ResCall<double> rc;
      rc.U = c->t0;
      rc.out = c->t1;
      FRX_TRY(launch_residual_f64(c->M, rc, s));
      rc.U = U;
      rc.out = c->t2;
      FRX_TRY(launch_residual_f64(c->M, rc, s));
      hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, c->sc + 11, 0.0);
      hipLaunchKernelGGL((k_fd_combine<double, double>), dim3(grid_for(n)), dim3(KR_THREADS), 0, s, (const double*)v,
                         c->t1, c->t2, nrm, (const double*)epsd, (const double*)(c->sc + 11), (double*)Jv, n,
                         (const int*)nullptr);
      FRX_TRY(hipGetLastError());
      // k_fd_combine computes sigma v - |v|(R1 - R0)/eps; with sigma = 0 negate
      hipLaunchKernelGGL(k_lincomb, dim3(grid_for(n)), dim3(KR_THREADS), 0, s, (double*)Jv, n, -1.0,
                         (const double*)Jv, 0.0, (const double*)nullptr, 0.0, (const double*)nullptr, 0.0,
                         (const double*)nullptr);
      FRX_TRY(hipGetLastError());
    }
    return FR_OK;
  });
}

fr_status fr_vjp(fr_ctx c, const double* U, const double* w, double* JTw, void* stream) {
  if (!c) return FR_E_INVALID;
  const size_t nb = sizeof(double) * c->ndof;
  if (!U || !w || !JTw || overlap(w, nb, JTw, nb) || overlap(U, nb, JTw, nb))
    return fail(c, FR_E_INVALID, "fr_vjp: bad arguments");
  return guarded(c, [&]() -> fr_status {
    FRX_TRY(launch_vjp(c->M, U, w, JTw, S(stream)));
    return FR_OK;
  });
}

fr_status gmres_stage_solve(fr_ctx c, const double* U, double shift, const double* F, double* dU,
                            const fr_gmres_opts* o, fr_gmres_stats* st, void* stream) {
  if (!c) return FR_E_INVALID;
  const size_t nb = sizeof(double) * c->ndof;
  if (!U || !F || !dU || !o || overlap(dU, nb, F, nb) || overlap(dU, nb, U, nb))
    return fail(c, FR_E_INVALID, "gmres_stage_solve: bad arguments");
  return guarded(c, [&]() -> fr_status {
    hipStream_t s = S(stream);
    fr_status r = gmres_solve(c, U, shift, F, dU, *o, st, s, nullptr);
    check_flag(c, s);
    if (r == FR_E_NOTCONVERGED) c->err = "gmres_stage_solve: iteration budget exhausted";
    return r;
  });
}

// Butcher tableaux of the ESDIRK schemes (section 2.3): explicit first
// stage, one diagonal coefficient w, stiffly accurate (b = last row).
// ESDIRK2: three stages, second order, w = 1 - sqrt(2)/2.  ESDIRK4: six
// stages, fourth order, w = 1/4, the scheme the paper cites from Bijl et al.
// (the implicit tableau of Kennedy and Carpenter's ARK4(3)6L[2]SA).
struct Esdirk {
  int s = 0;
  double A[6][6] = {};
};
Esdirk esdirk_scheme(int scheme) {
  Esdirk T;
  if (scheme == FR_ESDIRK2) {
    const double w = 1.0 - std::sqrt(2.0) / 2.0;
    T.s = 3;
    T.A[1][0] = T.A[1][1] = w;
    T.A[2][0] = T.A[2][1] = 0.5 * (1 - w);
    T.A[2][2] = w;
  } else if (scheme == FR_ESDIRK4) {
    T.s = 6;
    const double r[6][6] = {
        {0, 0, 0, 0, 0, 0},
        {0.25, 0.25, 0, 0, 0, 0},
        {8611.0 / 62500.0, -1743.0 / 31250.0, 0.25, 0, 0, 0},
        {5012029.0 / 34652500.0, -654441.0 / 2922500.0, 174375.0 / 388108.0, 0.25, 0, 0},
        {15267082809.0 / 155376265600.0, -71443401.0 / 120774400.0, 730878875.0 / 902184768.0,
         2285395.0 / 8070912.0, 0.25, 0},
        {82889.0 / 524892.0, 0.0, 15625.0 / 83664.0, 69875.0 / 102672.0, -2260.0 / 8211.0, 0.25}};
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) T.A[i][j] = r[i][j];
  }
  return T;
}

// out = base + sum_k coef[k] x[k] (terms with a zero coefficient skipped),
// three terms per pass
void accumulate(fr_ctx c, double* out, const double* base, const double* coef, const double* const* x, int cnt,
                hipStream_t s) {
  const double* cf[6];
  const double* xs[6];
  int m = 0;
  for (int k = 0; k < cnt; ++k)
    if (coef[k] != 0.0) {
      cf[m] = coef + k;
      xs[m++] = x[k];
    }
  const double* src = base;
  int k = 0;
  do {
    const double c1 = k < m ? *cf[k] : 0.0, c2 = k + 1 < m ? *cf[k + 1] : 0.0, c3 = k + 2 < m ? *cf[k + 2] : 0.0;
    lincomb(c, out, 1.0, src, c1, k < m ? xs[k] : nullptr, c2, k + 1 < m ? xs[k + 1] : nullptr, c3,
            k + 2 < m ? xs[k + 2] : nullptr, s);
    src = out;
    k += 3;
  } while (k < m);
}

fr_status esdirk_step(fr_ctx c, double* U, double dt, const fr_step_opts* o, fr_step_stats* st, void* stream) {
  if (!c) return FR_E_INVALID;
  if (!U || !o || !(dt > 0.0)) return fail(c, FR_E_INVALID, "esdirk_step: bad arguments");
  const Esdirk T = esdirk_scheme(o->scheme);
  if (!T.s) return fail(c, FR_E_INVALID, "esdirk_step: unknown scheme");
  const int last_stage = o->last_stage == 0 ? T.s : o->last_stage;
  if (last_stage < 2 || last_stage > T.s)
    return fail(c, FR_E_INVALID, "esdirk_step: last_stage must be 0 (the full step) or 2..stages");
  if (!(o->dtau_init > 0.0) || !(o->dtau_min > 0.0) || !(o->dtau_max >= o->dtau_init) ||
      !(o->dtau_min <= o->dtau_init) || !(o->tol_pseudo >= 0.0) || o->max_ptc_iter < 0)
    return fail(c, FR_E_INVALID,
                "esdirk_step: need 0 < dtau_min <= dtau_init <= dtau_max, tol_pseudo >= 0, max_ptc_iter >= 0");
  if (!c->es) return fail(c, FR_E_INVALID, "esdirk_step: the step workspace was not reserved (fr_reserve)");
  return guarded(c, [&]() -> fr_status {
    hipStream_t s = S(stream);
    const long n = c->ndof;
    double* qn = c->es;
    double* q = qn + n;
    double* rhs = q + n;
    double* F = rhs + n;
    double* dq = F + n;
    double* Rs = dq + n;  // up to 6 stage residuals
    const double(&A)[6][6] = T.A;
    const double w = A[1][1];
    const double* Rj[6];
    for (int j = 0; j < 6; ++j) Rj[j] = Rs + (size_t)j * n;
    fr_step_stats stats{0, 0, 0, 0, 0.0};
    FRX_TRY(hipMemcpyAsync(qn, U, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    FRX_TRY(hipMemcpyAsync(q, U, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    // the element-Jacobi preconditioner, evaluated once at the start of the
    // step (section 2.3) with sigma = 1/(omega dt) + 1/dtau_max
    if (o->gmres.precond) {
      if (c->pc_prec != o->gmres.precision || o->gmres.precond < 0 || o->gmres.precond > 2 ||
          (o->gmres.precond == 2 && c->pc_prec != FR_F32))
        throw StatusErr{FR_E_INVALID, "esdirk_step: no preconditioner storage in the GMRES precision (fr_reserve)"};
      pc_build(c, qn, 1.0 / (w * dt) + 1.0 / o->dtau_max, s, o->gmres.precond == 2);
    }
    ResCall<double> rc;
    rc.U = qn;
    rc.out = Rs;
    FRX_TRY(launch_residual_f64(c->M, rc, s));
    fr_status status = FR_OK;
    for (int i = 1; i < last_stage; ++i) {
      double cf[6];
      for (int j = 0; j < i; ++j) cf[j] = dt * A[i][j];
      accumulate(c, rhs, qn, cf, Rj, i, s);
      double dtau = o->dtau_init, nF0 = 0.0, nFprev = 0.0;
      double* Rq = Rs + (size_t)i * n;
      for (int m = 0;; ++m) {
        rc.U = q;
        rc.out = Rq;
        FRX_TRY(launch_residual_f64(c->M, rc, s));
        hipLaunchKernelGGL(k_stage_F, dim3(grid_for(n)), dim3(KR_THREADS), 0, s, (const double*)q, (const double*)Rq,
                           (const double*)rhs, 1.0 / (w * dt), F, n);
        FRX_TRY(hipGetLastError());
        // ||F|| and the non-physical flag in one round trip
        dot_to<double>(c, F, nullptr, c->sc + 15, nullptr, s);
        FRX_TRY(hipMemcpyAsync(c->hpin, c->sc + 15, sizeof(double), hipMemcpyDeviceToHost, s));
        FRX_TRY(hipMemcpyAsync(c->ipin, c->M.flag, sizeof(int), hipMemcpyDeviceToHost, s));
        FRX_TRY(hipStreamSynchronize(s));
        const double nF = std::sqrt(c->hpin[0]);
        if (c->ipin[0]) {
          hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, c->M.flag, 0);
          throw StatusErr{FR_E_NONPHYSICAL, "non-physical state (rho <= 0 or p <= 0) met in the residual"};
        }
        if (m == 0) nF0 = nF;
        else dtau = std::min(dtau * nFprev / nF, o->dtau_max);  // SER
        stats.final_rel_F = nF0 > 0 ? nF / nF0 : 0.0;
        if (nF <= o->tol_pseudo * nF0 || nF == 0.0) break;
        if (m >= o->max_ptc_iter) {
          status = FR_E_NOTCONVERGED;
          break;
        }
        while (true) {
          fr_gmres_stats gs;
          fr_status gr = gmres_solve(c, q, 1.0 / (w * dt) + 1.0 / dtau, F, dq, o->gmres, &gs, s, Rq, nF);
          stats.gmres_iterations += gs.iterations;
          if (gr == FR_OK) break;
          if (gr != FR_E_NOTCONVERGED) return gr;
          dtau *= 0.5;
          stats.halvings += 1;
          // dtau_min > 0 bounds the halvings of one iterate (by log2(dtau_max / dtau_min))
          if (dtau < o->dtau_min) {
            status = FR_E_NOTCONVERGED;
            break;
          }
        }
        if (status != FR_OK) break;
        lincomb(c, q, 1.0, q, 1.0, dq, 0, nullptr, 0, nullptr, s);
        nFprev = nF;
        stats.ptc_iterations += 1;
      }
      stats.stages += 1;
      if (status != FR_OK) break;
    }
    if (last_stage < T.s || status != FR_OK) {
      FRX_TRY(hipMemcpyAsync(U, q, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    } else {  // q^{n+1} = q^n + dt sum_j b_j R(q^j), b the last row
      double cf[6];
      for (int j = 0; j < T.s; ++j) cf[j] = dt * A[T.s - 1][j];
      accumulate(c, U, qn, cf, Rj, T.s, s);
    }
    FRX_TRY(hipStreamSynchronize(s));
    if (st) *st = stats;
    if (status != FR_OK) c->err = "esdirk_step: pseudo-transient continuation did not converge";
    return status;
  });
}

fr_status spectral_decay_indicator(fr_ctx c, const double* U, int32_t var, double* eta, double* eta_max,
                                   void* stream) {
  if (!c) return FR_E_INVALID;
  if (!U || !eta || !eta_max || var < 0 || var > 4) return fail(c, FR_E_INVALID, "spectral_decay_indicator: bad arguments");
  return guarded(c, [&]() -> fr_status {
    FRX_TRY(launch_indicator(c->M, U, var, eta, eta_max, S(stream)));
    return FR_OK;
  });
}

fr_status fr_select_degrees(fr_ctx c, const double* U, int32_t var, double nu_max, double nu_min, int32_t p_min,
                            int32_t p_max, int32_t eta_max_scope, int8_t* p_new, void* stream) {
  if (!c) return FR_E_INVALID;
  if (!U || !p_new || var < 0 || var > 4 || p_min < 1 || p_max > 5 || p_min > p_max || !(nu_min >= 0.0) ||
      !(nu_max >= nu_min) || (eta_max_scope != FR_ETA_MAX_ALL && eta_max_scope != FR_ETA_MAX_SAME_DEGREE))
    return fail(c, FR_E_INVALID, "fr_select_degrees: bad arguments");
  return guarded(c, [&]() -> fr_status {
    FRX_TRY(launch_select_degrees(c->M, U, var, nu_max, nu_min, p_min, p_max,
                                  eta_max_scope == FR_ETA_MAX_SAME_DEGREE ? 1 : 0, p_new, S(stream)));
    return FR_OK;
  });
}

fr_status fr_project(fr_ctx src, const double* U_src, fr_ctx dst, double* U_dst, void* stream) {
  if (!src || !dst) return FR_E_INVALID;
  if (!U_src || !U_dst || overlap(U_dst, sizeof(double) * dst->ndof, U_src, sizeof(double) * src->ndof))
    return fail(dst, FR_E_INVALID, "fr_project: bad arguments");
  if (src->M.E != dst->M.E || src->dev != dst->dev)
    return fail(dst, FR_E_INVALID, "fr_project: the two contexts must hold the same mesh on the same device");
  return guarded(dst, [&]() -> fr_status {
    FRX_TRY(launch_project(src->M, U_src, dst->M, U_dst, S(stream)));
    return FR_OK;
  });
}

fr_status fr_filter(fr_ctx c, const double* U, double* U_out, double alpha, int32_t p_from, void* stream) {
  if (!c) return FR_E_INVALID;
  if (!U || !U_out) return fail(c, FR_E_INVALID, "fr_filter: bad arguments");
  const size_t nb = sizeof(double) * c->ndof;
  if ((const double*)U_out != U && overlap(U_out, nb, U, nb))
    return fail(c, FR_E_INVALID, "fr_filter: U_out overlaps U without being U");
  if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(c, FR_E_INVALID, "fr_filter: alpha outside [0, 1]");
  if (p_from < 1 || p_from > NMAX - 1) return fail(c, FR_E_INVALID, "fr_filter: p_from outside 1..5");
  return guarded(c, [&]() -> fr_status {
    hipStream_t s = S(stream);
    if ((const double*)U_out != U)
      FRX_TRY(hipMemcpyAsync(U_out, U, sizeof(double) * c->ndof, hipMemcpyDeviceToDevice, s));
    FRX_TRY(launch_filter(c->M, U, U_out, alpha, p_from, s));
    return FR_OK;
  });
}

fr_status fr_set_launch(fr_ctx c, int32_t mode) {
  if (!c) return FR_E_INVALID;
  const int base = mode & ~(FR_LAUNCH_FACES_TWO_PASS | FR_LAUNCH_FACES_ONE_PASS);
  if ((base != FR_LAUNCH_PER_BUCKET && base != FR_LAUNCH_FUSED) ||
      ((mode & FR_LAUNCH_FACES_TWO_PASS) && (mode & FR_LAUNCH_FACES_ONE_PASS)))
    return fail(c, FR_E_INVALID, "fr_set_launch: mode");
  const bool fused = base == FR_LAUNCH_FUSED;
  bool changed = c->M.fused != fused;
  c->M.fused = fused;
  if (mode & (FR_LAUNCH_FACES_TWO_PASS | FR_LAUNCH_FACES_ONE_PASS)) {
    const bool two = (mode & FR_LAUNCH_FACES_TWO_PASS) != 0;
    for (int sk = 0; sk < SK_COUNT; ++sk) {
      changed = changed || c->M.split_faces[fused][sk] != two;
      c->M.split_faces[fused][sk] = two;
    }
  }
  if (!changed) return FR_OK;
  // the reserved graphs hold the old kernels: capture them again
  return guarded(c, [&]() -> fr_status {
    instantiate_graphs(c);
    return FR_OK;
  });
}

fr_status fr_check(fr_ctx c, int32_t* nonphysical, void* stream) {
  if (!c || !nonphysical) return FR_E_INVALID;
  return guarded(c, [&]() -> fr_status {
    hipStream_t s = S(stream);
    FRX_TRY(hipMemcpyAsync(c->ipin, c->M.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    FRX_TRY(hipStreamSynchronize(s));
    *nonphysical = c->ipin[0];
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, c->M.flag, 0);
    FRX_TRY(hipGetLastError());
    return FR_OK;
  });
}

// Launch-shape autotuner: for every scalar kind and every degree (pair)
// bucket, time the whole residual with each candidate elements-per-block
// (faces-per-block) of that bucket's kernel and keep the fastest.
fr_status fr_autotune(fr_ctx c, const double* U, void* stream) {
  if (!c || !U) return FR_E_INVALID;
  return guarded(c, [&]() -> fr_status {
    hipStream_t s = S(stream);
    const long n = c->ndof;
    hipLaunchKernelGGL((k_cast<double, float>), dim3(grid_for(n)), dim3(KR_THREADS), 0, s, U, c->uf, n);
    FRX_TRY(hipGetLastError());
    hipEvent_t e0, e1;
    FRX_TRY(hipEventCreate(&e0));
    FRX_TRY(hipEventCreate(&e1));
    auto run = [&](int sk) {
      if (sk == SK_F64) {
        ResCall<double> rc;
        rc.U = U;
        rc.out = c->t0;
        FRX_TRY(launch_residual_f64(c->M, rc, s));
      } else if (sk == SK_DUAL64) {
        ResCall<double> rc;
        rc.U = U;
        rc.V = U;
        rc.out = c->t0;
        FRX_TRY(launch_residual_dual64(c->M, rc, s));
      } else {
        ResCall<float> rc;
        rc.U = c->uf;
        rc.V = c->uf;
        rc.out = (float*)c->t1;
        FRX_TRY(launch_residual_dual32(c->M, rc, s));
      }
    };
    auto timed = [&](int sk) -> float {
      run(sk);
      FRX_TRY(hipEventRecord(e0, s));
      for (int r = 0; r < 5; ++r) run(sk);
      FRX_TRY(hipEventRecord(e1, s));
      FRX_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      FRX_TRY(hipEventElapsedTime(&ms, e0, e1));
      return ms;
    };
    const size_t lds_cap = 64 * 1024;
    const int cands[] = {1, 2, 4, 8, 16, 32, 64};
    for (int sk = 0; sk < SK_COUNT; ++sk) {
      const size_t sb = scalar_bytes(sk);
      for (ElemBucket& b : c->M.eb) {
        const int n3 = b.n * b.n * b.n;
        for (int kind = 0; kind < 2; ++kind) {
          int* slot = kind == 0 ? &b.epb_trace[sk] : &b.epb_div[sk];
          int best = *slot;
          float tbest = timed(sk);
          for (int e : cands) {
            const int tv = trace_lds_vals(c->M.physics == 1, b.n, (int)sb);
            const size_t lds = kind == 0 ? (size_t)e * tv * n3 * sb : (size_t)e * (5 * n3 + 30 * b.n * b.n) * sb;
            if (e == best || e * n3 > FRX_MAX_THREADS || lds > lds_cap || e > 2 * b.count) continue;
            *slot = e;
            const float t = timed(sk);
            if (t < tbest) {
              tbest = t;
              best = e;
            }
          }
          *slot = best;
        }
      }
      for (FaceBucket& f : c->M.fb) {
        const int nh2 = f.nh * f.nh;
        const size_t per = f.nl < f.nh ? (size_t)(20 * f.nl * f.nl + 10 * nh2) * sb : 0;
        int best = f.fpb[sk];
        float tbest = timed(sk);
        for (int e : cands) {
          if (e == best || e * nh2 > FRX_MAX_THREADS || (size_t)e * per > lds_cap || e > 2 * f.count) continue;
          f.fpb[sk] = e;
          const float t = timed(sk);
          if (t < tbest) {
            tbest = t;
            best = e;
          }
        }
        f.fpb[sk] = best;
      }
    }
    // Fused plans: for every scalar kind, stage and bucket code (degree, or
    // degree pair of interior faces), the items per tile among the largest
    // that fits (256 threads, the stage's LDS cap), its half and its quarter
    // that times fastest in the fused launch, one code at a time with the
    // others at their current choice
    {
      const bool fused0 = c->M.fused;
      c->M.fused = true;
      const bool ns = c->M.physics == 1;
      for (int sk = 0; sk < SK_COUNT; ++sk)
        for (int st = 0; st < 3; ++st) {
          std::vector<int> codes;
          if (st != 1)
            for (auto& kv : c->erange) codes.push_back(kv.first);
          else
            for (auto& fr : c->frange)
              if (std::get<0>(fr) < 64) codes.push_back(std::get<0>(fr));
          for (int code : codes) {
            const int mx = max_items(ns, sk, st, code);
            auto it = c->shape[sk][st].find(code);
            int best = it != c->shape[sk][st].end() ? it->second : mx;
            float tbest = timed(sk);
            for (int k : {mx, mx / 2, mx / 4}) {
              if (k < 1 || k == best) continue;
              c->shape[sk][st][code] = k;
              plan_stage(c, sk, st);
              const float t = timed(sk);
              if (t < tbest) {
                tbest = t;
                best = k;
              }
            }
            c->shape[sk][st][code] = best;
            plan_stage(c, sk, st);
          }
        }
      c->M.fused = fused0;
    }
    // Navier-Stokes face stage in one or two passes, per launch mode and
    // scalar kind: the faster of the two
    if (c->M.physics == 1) {
      const bool fused0 = c->M.fused;
      for (int fm = 0; fm < 2; ++fm) {
        c->M.fused = fm == 1;
        for (int sk = 0; sk < SK_COUNT; ++sk) {
          c->M.split_faces[fm][sk] = false;
          const float t1 = timed(sk);
          c->M.split_faces[fm][sk] = true;
          const float t2 = timed(sk);
          c->M.split_faces[fm][sk] = t2 < t1;
        }
      }
      c->M.fused = fused0;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the reserved graphs hold the old shapes: capture them again
    instantiate_graphs(c);
    return FR_OK;
  });
}

fr_status fr_profile(fr_ctx c, const double* U, int32_t op, int32_t reps, fr_kernel_time* out, int32_t max_out,
                     int32_t* n_out, void* stream) {
  if (!c || !U || !out || !n_out || reps < 1 || op < 0 || op > 3) return c ? fail(c, FR_E_INVALID, "fr_profile: bad arguments") : FR_E_INVALID;
  return guarded(c, [&]() -> fr_status {
    hipStream_t s = S(stream);
    const long n = c->ndof;
    hipLaunchKernelGGL((k_cast<double, float>), dim3(grid_for(n)), dim3(KR_THREADS), 0, s, U, c->uf, n);
    FRX_TRY(hipGetLastError());
    ProfHook P;
    auto run = [&]() {
      if (op == 0) {
        ResCall<double> rc;
        rc.U = U;
        rc.out = c->t0;
        FRX_TRY(launch_residual_f64(c->M, rc, s));
      } else if (op == 1 || op == 3) {
        ResCall<double> rc;
        rc.U = U;
        rc.V = U;
        rc.out = c->t0;
        if (op == 3) rc.out_val = c->t2;  // the one-pass residual and tangent
        FRX_TRY(launch_residual_dual64(c->M, rc, s));
      } else {
        ResCall<float> rc;
        rc.U = c->uf;
        rc.V = c->uf;
        rc.out = (float*)c->t1;
        FRX_TRY(launch_residual_dual32(c->M, rc, s));
      }
    };
    run();  // warm-up, untimed
    c->M.prof = &P;
    try {
      for (int r = 0; r < reps; ++r) run();
    } catch (...) {
      c->M.prof = nullptr;
      throw;
    }
    c->M.prof = nullptr;
    FRX_TRY(hipStreamSynchronize(s));
    const size_t per = P.recs.size() / reps;
    int k = 0;
    for (size_t i = 0; i < per && k < max_out; ++i, ++k) {
      double tot = 0.0;
      for (int r = 0; r < reps; ++r) {
        float ms = 0.f;
        FRX_TRY(hipEventElapsedTime(&ms, P.recs[r * per + i].a, P.recs[r * per + i].b));
        tot += ms;
      }
      const auto& R = P.recs[i];
      std::snprintf(out[k].stage, sizeof(out[k].stage), "%s", R.stage);
      out[k].n_lo = R.nl;
      out[k].n_hi = R.nh;
      out[k].units = R.units;
      out[k].ms = tot / reps;
    }
    for (auto& R : P.recs) {
      (void)hipEventDestroy(R.a);
      (void)hipEventDestroy(R.b);
    }
    *n_out = k;
    return FR_OK;
  });
}

fr_status fr_precond_build(fr_ctx c, const double* U, double sigma, int32_t precision, void* stream) {
  if (!c) return FR_E_INVALID;
  if (!U || !(sigma > 0.0) || (precision != FR_F64 && precision != FR_F32 && precision != FR_PC_F16))
    return fail(c, FR_E_INVALID, "fr_precond_build: bad arguments");
  if (c->pc_prec != (precision == FR_PC_F16 ? FR_F32 : precision))
    return fail(c, FR_E_INVALID, "fr_precond_build: no preconditioner storage in this precision (fr_reserve)");
  return guarded(c, [&]() -> fr_status {
    c->pc_built = false;
    pc_build(c, U, sigma, S(stream), precision == FR_PC_F16);
    return FR_OK;
  });
}

fr_status fr_precond_apply(fr_ctx c, const double* x, double* y, void* stream) {
  if (!c) return FR_E_INVALID;
  const size_t nb = sizeof(double) * c->ndof;
  if (!x || !y || ((const void*)x != (const void*)y && overlap(x, nb, y, nb)))
    return fail(c, FR_E_INVALID, "fr_precond_apply: bad arguments");
  if (!c->pc_built) return fail(c, FR_E_INVALID, "fr_precond_apply: no preconditioner built (fr_precond_build)");
  return guarded(c, [&]() -> fr_status {
    hipStream_t s = S(stream);
    if (x != y) FRX_TRY(hipMemcpyAsync(y, x, nb, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, c->ist + 5, c->pc_half ? 2 : 1);
    pc_apply<double>(c, y, nullptr, s);
    return FR_OK;
  });
}

fr_status fr_launch_shapes(fr_ctx c, int32_t kind, int32_t* out, int32_t max_out, int32_t* n_out) {
  if (!c || !n_out || max_out < 0 || (max_out > 0 && !out) || kind < 0 || kind >= SK_COUNT)
    return c ? fail(c, FR_E_INVALID, "fr_launch_shapes: bad arguments") : FR_E_INVALID;
  const bool ns = c->M.physics == 1;
  int k = 0;
  for (int st = 0; st < 3; ++st) {
    std::vector<int> codes;
    if (st != 1)
      for (auto& kv : c->erange) codes.push_back(kv.first);
    else
      for (auto& fr : c->frange)
        if (std::get<0>(fr) < 64) codes.push_back(std::get<0>(fr));
    for (int code : codes) {
      if (k < max_out) {
        auto it = c->shape[kind][st].find(code);
        out[3 * k] = st;
        out[3 * k + 1] = code;
        out[3 * k + 2] = it != c->shape[kind][st].end() ? it->second : max_items(ns, kind, st, code);
      }
      ++k;
    }
  }
  *n_out = std::min(k, max_out);
  return FR_OK;
}

const char* fr_last_error(fr_ctx c) { return c ? c->err.c_str() : g_create_error.c_str(); }

}  // extern "C"
