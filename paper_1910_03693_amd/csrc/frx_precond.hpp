// Element-Jacobi preconditioner of section 2.3: the diagonal blocks of
// (sigma I - dR/dq), sigma = 1/(omega dt) + 1/dtau_max, one dense block per
// element (N = 5 (p+1)^3 rows), factored once and applied to every Krylov
// vector (left preconditioning).
//
// Assembly: the columns of the element blocks come from exact tangent
// products.  The elements are coloured so that no two face neighbours share a
// colour; seeding DOF j of every element of one colour gives, in those
// elements' own rows, column j of their diagonal blocks (the residual of an
// element depends on its own and its face neighbours' DOF only).
// Factorisation: LU with partial pivoting, one 256-thread block per element,
// the matrix column-major in device memory.  Apply: permutation, forward and
// backward substitution, one block per element, in place.
#pragma once
#include <hip/hip_runtime.h>

namespace frx {

// element record of the preconditioner: (element, first solution point, n = p + 1, 0)
struct PcDev {
  const int4* recs;    // [E]
  const long* boff;    // [E] first entry of each block
  const int* poff;     // [E] first pivot of each block
};

__device__ __forceinline__ int pc_rows(int n) { return 5 * n * n * n; }
// DOF j of an element (variable-major inside the element: j = v n^3 + k) in
// the state layout U[v][sp]
__device__ __forceinline__ long pc_dof(int j, int n, int sp0, int nsp) {
  const int n3 = n * n * n;
  return (long)(j / n3) * nsp + sp0 + (j % n3);
}

// Seed of one assembly product: over the elements of one colour, clear the
// previous column's DOF and set column j's (if the element has that many).
template <class TV>
__global__ void __launch_bounds__(256) k_pc_seed(TV* __restrict__ V, int nsp, const int4* __restrict__ crecs, int ncol,
                                                int j_prev, int j) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncol) return;
  const int4 r = crecs[t];
  const int N = pc_rows(r.z);
  if (j_prev >= 0 && j_prev < N) V[pc_dof(j_prev, r.z, r.y, nsp)] = TV(0);
  if (j >= 0 && j < N) V[pc_dof(j, r.z, r.y, nsp)] = TV(1);
}

// Column j of the blocks of one colour's elements: sigma e_j - (J v)_e, v
// the seed; one block of threads per element, rows over the threads.
template <class TV, class TB>
__global__ void __launch_bounds__(256) k_pc_extract(const TV* __restrict__ Jv, int nsp, const int4* __restrict__ crecs,
                                                   const int* __restrict__ cidx, int j, double sigma,
                                                   const long* __restrict__ boff, TB* __restrict__ blocks) {
  const int4 r = crecs[blockIdx.x];
  const int N = pc_rows(r.z);
  if (j >= N) return;
  TB* A = blocks + boff[cidx[blockIdx.x]] + (long)j * N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const double jv = (double)Jv[pc_dof(i, r.z, r.y, nsp)];
    A[i] = (TB)((i == j ? sigma : 0.0) - jv);
  }
}

// LU factorisation with partial pivoting of every element block, in place:
// P A = L U with unit lower L; piv[k] = the row swapped with row k at step k.
// A zero pivot column (a singular block) sets *flag.
template <class TB>
__global__ void __launch_bounds__(256) k_pc_lu(TB* __restrict__ blocks, PcDev pc, int* __restrict__ piv,
                                              int* __restrict__ flag) {
  __shared__ double red_v[256];
  __shared__ int red_i[256];
  __shared__ TB rowk[5 * 6 * 6 * 6];
  const int4 r = pc.recs[blockIdx.x];
  const int N = pc_rows(r.z);
  TB* A = blocks + pc.boff[blockIdx.x];
  int* P = piv + pc.poff[blockIdx.x];
  const int tid = threadIdx.x;
  for (int k = 0; k < N; ++k) {
    // pivot: the largest |a_ik|, i >= k (the smallest index among equals)
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < N; i += blockDim.x) {
      const double v = fabs((double)A[i + (long)k * N]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    red_v[tid] = best;
    red_i[tid] = bi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) {
        const double a = red_v[tid], b = red_v[tid + s];
        if (b > a || (b == a && red_i[tid + s] < red_i[tid])) {
          red_v[tid] = b;
          red_i[tid] = red_i[tid + s];
        }
      }
      __syncthreads();
    }
    const int p = red_i[0];
    const bool singular = !(red_v[0] > 0.0);
    __syncthreads();
    if (tid == 0) {
      P[k] = p;
      if (singular) *flag = 1;
    }
    if (p != k)
      for (int j = tid; j < N; j += blockDim.x) {
        const TB t = A[k + (long)j * N];
        A[k + (long)j * N] = A[p + (long)j * N];
        A[p + (long)j * N] = t;
      }
    __syncthreads();
    for (int j = k + 1 + tid; j < N; j += blockDim.x) rowk[j] = A[k + (long)j * N];
    __syncthreads();
    const TB pivot = A[k + (long)k * N];
    const TB inv = singular ? TB(0) : TB(1) / pivot;
    // multipliers and the rank-1 update of the trailing rows, a row per thread
    for (int i = k + 1 + tid; i < N; i += blockDim.x) {
      const TB l = A[i + (long)k * N] * inv;
      A[i + (long)k * N] = l;
      for (int j = k + 1; j < N; ++j) A[i + (long)j * N] -= l * rowk[j];
    }
    __syncthreads();
  }
}

// x_e <- P_e^{-1} x_e for every element, in place (x: the Krylov vector, TV
// storage; the substitution runs in TB).  *on == 0 leaves x unchanged (one
// captured graph serves the preconditioned and the plain solves); *done != 0
// returns at once, as every kernel of a captured Arnoldi step.
template <class TV, class TB>
__global__ void __launch_bounds__(256) k_pc_apply(TV* __restrict__ x, int nsp, const TB* __restrict__ blocks, PcDev pc,
                                                 const int* __restrict__ piv, const int* __restrict__ on,
                                                 const int* __restrict__ done) {
  if (!*on || (done && *done)) return;
  __shared__ TB y[5 * 6 * 6 * 6];
  const int4 r = pc.recs[blockIdx.x];
  const int N = pc_rows(r.z);
  const TB* A = blocks + pc.boff[blockIdx.x];
  const int* P = piv + pc.poff[blockIdx.x];
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += blockDim.x) y[i] = (TB)x[pc_dof(i, r.z, r.y, nsp)];
  __syncthreads();
  if (tid == 0)
    for (int k = 0; k < N; ++k) {  // the row swaps, in the order of the factorisation
      const int p = P[k];
      if (p != k) {
        const TB t = y[k];
        y[k] = y[p];
        y[p] = t;
      }
    }
  __syncthreads();
  // forward: L (unit diagonal), column by column
  for (int k = 0; k < N - 1; ++k) {
    const TB yk = y[k];
    for (int i = k + 1 + tid; i < N; i += blockDim.x) y[i] -= A[i + (long)k * N] * yk;
    __syncthreads();
  }
  // backward: U, column by column from the last
  for (int k = N - 1; k >= 0; --k) {
    if (tid == 0) y[k] /= A[k + (long)k * N];
    __syncthreads();
    const TB yk = y[k];
    for (int i = tid; i < k; i += blockDim.x) y[i] -= A[i + (long)k * N] * yk;
    __syncthreads();
  }
  for (int i = tid; i < N; i += blockDim.x) x[pc_dof(i, r.z, r.y, nsp)] = (TV)y[i];
}

}  // namespace frx
