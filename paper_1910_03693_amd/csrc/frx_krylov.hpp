// Device kernels of the matrix-free restarted GMRES (section 2.3 of the paper:
// PETSc GMRES with a user mat-vec; here the Krylov solver runs on the GPU).
//
// Arnoldi with classical Gram-Schmidt applied twice (CGS2): each pass is one
// multi-dot (deterministic two-level reduction, FP64 accumulation whatever the
// storage type of the basis) and one multi-axpy.  The Hessenberg matrix,
// Givens rotations, residual estimate and least-squares solve stay in FP64 and
// on the device; a device flag marks convergence so that the kernels of the
// remaining iterations of a captured cycle return at once.
#pragma once
#include <hip/hip_runtime.h>

namespace frx {

constexpr int KR_THREADS = 256;
constexpr int KR_VB = 8;  // vectors per multi-dot block row

struct GmresDev {
  double* H;      // [(m+1) x m] row-major, H[i*m + j]
  double* cs;     // [m]
  double* sn;     // [m]
  double* g;      // [m+1]
  double* y;      // [m]
  double* part;   // [(m+1) x nblk] multi-dot partials
  double* hbuf;   // [m+1] current multi-dot result
  double* sc;     // scalars: 0 beta, 1 ||F||, 2 tol, 3 residual estimate, 4 1/h_{j+1,j}, 5 sigma
  int* ist;       // ints: 0 done flag, 1 iterations of this cycle, 2 total iterations, 3 iteration budget,
                  // 4 length of this cycle (<= m), 5 preconditioner on, 6 one-pass Gram-Schmidt
  int m;          // leading dimension of H: the largest cycle the workspace holds
  int nblk;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// block-wide sum over KR_THREADS threads (4 wavefronts), result in thread 0
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < KR_THREADS / 64; ++i) s += sh[i];
  __syncthreads();
  return s;
}

// part[i * nblk + blockIdx.x] = sum over this block's grid-stride share of
// w * V_i for i in [y0, y0 + KR_VB) (blockIdx.y selects y0).  If V == nullptr
// the second operand is w itself (a norm).
template <class TV, class TW>
__global__ void __launch_bounds__(KR_THREADS) k_multidot(const TV* __restrict__ V, long ldv, int nv,
                                                        const TW* __restrict__ w, long n, double* __restrict__ part,
                                                        int nblk, const int* __restrict__ done) {
  if (done && *done) return;
  __shared__ double sh[KR_THREADS / 64];
  const int y0 = blockIdx.y * KR_VB;
  const int cnt = V ? min(KR_VB, nv - y0) : 1;
  double s[KR_VB];
#pragma unroll
  for (int i = 0; i < KR_VB; ++i) s[i] = 0.0;
  for (long t = (long)blockIdx.x * KR_THREADS + threadIdx.x; t < n; t += (long)nblk * KR_THREADS) {
    const double wt = (double)w[t];
    if (!V) {
      s[0] += wt * wt;
      continue;
    }
#pragma unroll
    for (int i = 0; i < KR_VB; ++i)
      if (i < cnt) s[i] += wt * (double)V[(long)(y0 + i) * ldv + t];
  }
#pragma unroll
  for (int i = 0; i < KR_VB; ++i) {
    if (i >= cnt) break;
    const double r = block_sum(s[i], sh);
    if (threadIdx.x == 0) part[(long)(y0 + i) * nblk + blockIdx.x] = r;
  }
}

// out[i] = sum_b part[i * nblk + b]  (one block per entry, fixed order)
__global__ void __launch_bounds__(KR_THREADS) k_reduce(const double* __restrict__ part, int nblk, double* out,
                                                      const int* __restrict__ done) {
  if (done && *done) return;
  __shared__ double sh[KR_THREADS / 64];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += KR_THREADS) s += part[(long)blockIdx.x * nblk + b];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// w -= sum_{i < nv} h[i] V_i   (FP64 arithmetic, stored as TW)
template <class TV, class TW>
__global__ void __launch_bounds__(KR_THREADS) k_multiaxpy(const TV* __restrict__ V, long ldv, int nv,
                                                         const double* __restrict__ h, TW* __restrict__ w, long n,
                                                         const int* __restrict__ done) {
  if (done && *done) return;
  for (long t = (long)blockIdx.x * KR_THREADS + threadIdx.x; t < n; t += (long)gridDim.x * KR_THREADS) {
    double acc = (double)w[t];
    for (int i = 0; i < nv; ++i) acc -= h[i] * (double)V[(long)i * ldv + t];
    w[t] = (TW)acc;
  }
}

// x *= *sptr in place
template <class TV>
__global__ void __launch_bounds__(KR_THREADS) k_scale_inplace(TV* __restrict__ x, long n,
                                                             const double* __restrict__ sptr,
                                                             const int* __restrict__ done) {
  if (done && *done) return;
  const double s = *sptr;
  for (long t = (long)blockIdx.x * KR_THREADS + threadIdx.x; t < n; t += (long)gridDim.x * KR_THREADS)
    x[t] = (TV)((double)x[t] * s);
}

// x += sum_{i < k} y[i] V_i  with k read from the device
template <class TV>
__global__ void __launch_bounds__(KR_THREADS) k_update_x(const TV* __restrict__ V, long ldv, const double* __restrict__ y,
                                                        const int* __restrict__ kptr, double* __restrict__ x, long n) {
  const int k = *kptr;
  for (long t = (long)blockIdx.x * KR_THREADS + threadIdx.x; t < n; t += (long)gridDim.x * KR_THREADS) {
    double acc = x[t];
    for (int i = 0; i < k; ++i) acc += y[i] * (double)V[(long)i * ldv + t];
    x[t] = acc;
  }
}

// dst = src * scale, scale = *sptr (or 1 / *sptr if inv), cast to TD
template <class TS, class TD>
__global__ void __launch_bounds__(KR_THREADS) k_scale(const TS* __restrict__ src, TD* __restrict__ dst, long n,
                                                     const double* __restrict__ sptr, int inv,
                                                     const int* __restrict__ done) {
  if (done && *done) return;
  const double s = inv ? 1.0 / *sptr : *sptr;
  for (long t = (long)blockIdx.x * KR_THREADS + threadIdx.x; t < n; t += (long)gridDim.x * KR_THREADS)
    dst[t] = (TD)((double)src[t] * s);
}

// Start of a cycle: beta = sqrt(dot), g = (beta, 0, ...), done = (beta <= tol ||F||).
__global__ void k_cycle_start(GmresDev G, const double* __restrict__ dot) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double beta = sqrt(*dot);
  G.sc[0] = beta;
  G.sc[3] = beta;
  G.sc[4] = beta > 0.0 ? 1.0 / beta : 0.0;
  for (int i = 0; i <= G.m; ++i) G.g[i] = 0.0;
  G.g[0] = beta;
  G.ist[1] = 0;
  G.ist[0] = (beta <= G.sc[2] * G.sc[1] || G.ist[2] >= G.ist[3]) ? 1 : 0;
}

// Column j of H from the two Gram-Schmidt passes (h1 + h2) and the squared
// norm of the orthogonalised vector; Givens rotation; residual estimate
// |g_{j+1}|; convergence or budget check; 1/h_{j+1,j} for the scaling of the
// new vector.  One thread.
__device__ __forceinline__ void givens_step(const GmresDev& G, int j, const double* __restrict__ h1,
                                            const double* __restrict__ h2, double nrm2) {
  if (G.ist[0]) return;
  const int m = G.m;
  for (int i = 0; i <= j; ++i) G.H[i * m + j] = h1[i] + h2[i];
  const double hn = sqrt(nrm2);
  G.H[(j + 1) * m + j] = hn;
  for (int i = 0; i < j; ++i) {
    const double a = G.H[i * m + j], b = G.H[(i + 1) * m + j];
    G.H[i * m + j] = G.cs[i] * a + G.sn[i] * b;
    G.H[(i + 1) * m + j] = -G.sn[i] * a + G.cs[i] * b;
  }
  const double a = G.H[j * m + j], b = hn;
  const double den = sqrt(a * a + b * b);
  const double c = den > 0.0 ? a / den : 1.0, s = den > 0.0 ? b / den : 0.0;
  G.cs[j] = c;
  G.sn[j] = s;
  G.H[j * m + j] = den;
  G.H[(j + 1) * m + j] = 0.0;
  G.g[j + 1] = -s * G.g[j];
  G.g[j] = c * G.g[j];
  const double res = fabs(G.g[j + 1]);
  G.sc[3] = res;
  G.sc[4] = hn > 0.0 ? 1.0 / hn : 0.0;
  G.ist[1] = j + 1;
  G.ist[2] += 1;
  if (res <= G.sc[2] * G.sc[1] || hn == 0.0 || G.ist[2] >= G.ist[3] || j + 1 >= G.ist[4]) G.ist[0] = 1;
}

__global__ void k_givens(GmresDev G, int j, const double* __restrict__ h1, const double* __restrict__ h2,
                         const double* __restrict__ nrm2) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  givens_step(G, j, h1, h2, *nrm2);
}

// ---------------------------------------------- fused Gram-Schmidt passes
// For NV <= 32 basis vectors (one instantiation per NV, so that no load sits
// behind a branch) every thread keeps the partial sums of all NV dots in
// registers, and one launch reads w and each V_i once (k_multidot splits the
// vectors over block rows and reads w once per row).
//  MODE 0: sums V_i . w                                     (first pass dots)
//  MODE 1: w -= sum_i h_i V_i (stored as TV); sums V_i . w   (first pass
//          update fused with the second pass dots)
//  MODE 2: out = w - sum_i h_i V_i (stored as TV); sum |out|^2
// With *one != 0 (one-pass classical Gram-Schmidt) MODE 1 does nothing and
// MODE 2 subtracts h1 (the first pass coefficients, hx) instead of h.
// Each block writes its partial sums to part[i * nblk + blockIdx.x];
// k_gs_reduce adds them up in a fixed order.  (A last-block reduction inside
// k_gs would need a device-scope fence per block, which costs an L2
// write-back each on this chip.)
template <class TV, int NV, int MODE>
__global__ void __launch_bounds__(KR_THREADS) k_gs(const TV* __restrict__ V, long ldv, const double* __restrict__ h,
                                                  TV* w, TV* __restrict__ out, long n, double* __restrict__ part,
                                                  const int* __restrict__ done, const double* __restrict__ hx,
                                                  const int* __restrict__ one) {
  if (done && *done) return;
  if (MODE == 1 && one && *one) return;
  constexpr int NS = MODE == 2 ? 1 : NV;
  __shared__ double sh[KR_THREADS / 64][NS];
  __shared__ double hs[NV];
  const int nblk = gridDim.x;
  if (MODE != 0) {
    if (threadIdx.x < NV) hs[threadIdx.x] = (MODE == 2 && one && *one) ? hx[threadIdx.x] : h[threadIdx.x];
    __syncthreads();
  }
  double s[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) s[i] = 0.0;
  // grid-stride rows, UR per trip so that the loads of all of them are in
  // flight together; the rows are still accumulated in grid-stride order
  constexpr int UR = NV <= 2 ? 8 : (NV <= 4 ? 4 : (NV <= 16 ? 2 : 1));
  const long stride = (long)nblk * KR_THREADS;
  for (long t = (long)blockIdx.x * KR_THREADS + threadIdx.x; t < n; t += UR * stride) {
    TV v[UR][NV];
    double a[UR];
    bool in[UR];
    long tr[UR];
#pragma unroll
    for (int r = 0; r < UR; ++r) {
      in[r] = t + r * stride < n;
      tr[r] = in[r] ? t + r * stride : t;  // a valid row; its values are not used
    }
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int r = 0; r < UR; ++r) v[r][i] = V[(long)i * ldv + tr[r]];
#pragma unroll
    for (int r = 0; r < UR; ++r) a[r] = (double)w[tr[r]];
    // keep the scheduler from interleaving the loads with the arithmetic, so
    // that all of them are in flight at once
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < UR; ++r) {
      if (MODE != 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) a[r] -= hs[i] * (double)v[r][i];
        const TV st = (TV)a[r];
        if (in[r]) {
          if (MODE == 1) w[tr[r]] = st;
          else out[tr[r]] = st;
        }
        a[r] = (double)st;
      }
      if (!in[r]) a[r] = 0.0;
      if (MODE == 2) {
        s[0] += a[r] * a[r];
      } else {
#pragma unroll
        for (int i = 0; i < NV; ++i) s[i] += a[r] * (double)v[r][i];
      }
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const double r = wave_sum(s[i]);
    if (lane == 0) sh[wv][i] = r;
  }
  __syncthreads();
  if (threadIdx.x < NS) {
    double r = 0.0;
#pragma unroll
    for (int k = 0; k < KR_THREADS / 64; ++k) r += sh[k][threadIdx.x];
    part[(long)threadIdx.x * nblk + blockIdx.x] = r;
  }
}

// Final sums of the block partials of k_gs: block i adds up entry i in a fixed
// order; after the norm pass (givens != 0, one entry) the Givens step of
// column j follows.
__global__ void __launch_bounds__(KR_THREADS) k_gs_reduce(const double* __restrict__ part, int nblk,
                                                         double* __restrict__ hout, int givens, GmresDev G, int j,
                                                         const double* __restrict__ h1,
                                                         const double* __restrict__ h2,
                                                         const int* __restrict__ done,
                                                         const int* __restrict__ zero) {
  if (done && *done) return;
  if (zero && *zero) {  // the second pass skipped: its coefficients are 0
    if (threadIdx.x == 0) hout[blockIdx.x] = 0.0;
    return;
  }
  __shared__ double sh[KR_THREADS / 64];
  double r = 0.0;
  for (int b = threadIdx.x; b < nblk; b += KR_THREADS) r += part[(long)blockIdx.x * nblk + b];
  r = block_sum(r, sh);
  if (threadIdx.x == 0) {
    hout[blockIdx.x] = r;
    if (givens) givens_step(G, j, h1, h2, r);
  }
}

// y = H(0:k, 0:k)^{-1} g(0:k) by back substitution, k = iterations of the cycle
__global__ void k_backsolve(GmresDev G) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int k = G.ist[1], m = G.m;
  for (int i = k - 1; i >= 0; --i) {
    double s = G.g[i];
    for (int l = i + 1; l < k; ++l) s -= G.H[i * m + l] * G.y[l];
    G.y[i] = s / G.H[i * m + i];
  }
}

// ------------------------------------------------------------ vector kernels
// F = (rhs - q) / (omega dt) + R   (eq. ESDIRK_conservative)
__global__ void __launch_bounds__(KR_THREADS) k_stage_F(const double* __restrict__ q, const double* __restrict__ R,
                                                       const double* __restrict__ rhs, double inv_wdt,
                                                       double* __restrict__ F, long n) {
  for (long t = (long)blockIdx.x * KR_THREADS + threadIdx.x; t < n; t += (long)gridDim.x * KR_THREADS)
    F[t] = (rhs[t] - q[t]) * inv_wdt + R[t];
}

// out = c0 x0 + c1 x1 + c2 x2 + c3 x3 (null inputs skipped)
__global__ void __launch_bounds__(KR_THREADS) k_lincomb(double* __restrict__ out, long n, double c0,
                                                       const double* x0, double c1, const double* x1, double c2,
                                                       const double* x2, double c3, const double* x3) {
  for (long t = (long)blockIdx.x * KR_THREADS + threadIdx.x; t < n; t += (long)gridDim.x * KR_THREADS) {
    double s = c0 * x0[t];
    if (x1) s += c1 * x1[t];
    if (x2) s += c2 * x2[t];
    if (x3) s += c3 * x3[t];
    out[t] = s;
  }
}

// finite-difference perturbation Up = U + eps * v / ||v||  (||v||^2 and eps
// on the device, so that a captured graph reads the current step)
template <class TV>
__global__ void __launch_bounds__(KR_THREADS) k_fd_perturb(const double* __restrict__ U, const TV* __restrict__ v,
                                                          const double* __restrict__ nrm2,
                                                          const double* __restrict__ epsp, double* __restrict__ Up,
                                                          long n, const int* __restrict__ done) {
  if (done && *done) return;
  const double nv = sqrt(*nrm2);
  const double s = nv > 0.0 ? *epsp / nv : 0.0;
  for (long t = (long)blockIdx.x * KR_THREADS + threadIdx.x; t < n; t += (long)gridDim.x * KR_THREADS)
    Up[t] = U[t] + s * (double)v[t];
}

// out = sigma v - ||v|| (R1 - R0) / eps   (the finite-difference operator)
template <class TV, class TO>
__global__ void __launch_bounds__(KR_THREADS) k_fd_combine(const TV* __restrict__ v, const double* __restrict__ R1,
                                                          const double* __restrict__ R0,
                                                          const double* __restrict__ nrm2,
                                                          const double* __restrict__ epsp,
                                                          const double* __restrict__ sigma, TO* __restrict__ out,
                                                          long n, const int* __restrict__ done) {
  if (done && *done) return;
  const double nv = sqrt(*nrm2);
  const double sg = *sigma, eps = *epsp;
  for (long t = (long)blockIdx.x * KR_THREADS + threadIdx.x; t < n; t += (long)gridDim.x * KR_THREADS)
    out[t] = (TO)(sg * (double)v[t] - nv * (R1[t] - R0[t]) / eps);
}

template <class TS, class TD>
__global__ void __launch_bounds__(KR_THREADS) k_cast(const TS* __restrict__ s, TD* __restrict__ d, long n) {
  for (long t = (long)blockIdx.x * KR_THREADS + threadIdx.x; t < n; t += (long)gridDim.x * KR_THREADS) d[t] = (TD)s[t];
}

// *out = eps sqrt(1 + sqrt(*nrm2)): the finite-difference step scaled to the
// state (Walker and Pernice's choice), *nrm2 = ||U||^2
__global__ void k_fd_scaled_eps(const double* __restrict__ nrm2, double eps, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = eps * sqrt(1.0 + sqrt(*nrm2));
}

__global__ void k_set_scalar(double* p, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}
__global__ void k_set_int(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}
__global__ void __launch_bounds__(KR_THREADS) k_fill(double* p, long n, double v) {
  for (long t = (long)blockIdx.x * KR_THREADS + threadIdx.x; t < n; t += (long)gridDim.x * KR_THREADS) p[t] = v;
}

}  // namespace frx
