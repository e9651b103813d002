// Spectral-decay smoothness indicator (section 3.1 of the paper, after
// Persson & Peraire): for one variable s of every element
//   eta = ||s_p - s_{p-1}|| / ||s_p||,
// with the paper's |J|-weighted Gauss "L2" norm (a weighted mean of squares;
// the normalising sums cancel in the ratio) and s_{p-1} the projection onto
// tensor degree p-1, i.e. the Legendre modes whose indices are all below p.
// Modal coefficients use the exactness of Gauss quadrature:
//   c_m = (2m+1)/2 sum_k w_k P_m(x_k) s_k  per direction.
#pragma once
#include "frx_device.hpp"

namespace frx {

// Block: epb elements x N^3 threads; LDS: two regions of N^3 doubles per element.
template <int N>
__global__ void __launch_bounds__(1024) k_indicator(const double* __restrict__ U, int nsp, int var,
                                                   const int* __restrict__ sp_off, const double* __restrict__ geo,
                                                   const int* __restrict__ elems, int nel, int epb,
                                                   double* __restrict__ eta) {
  constexpr int N2 = N * N, N3 = N2 * N;
  extern __shared__ __align__(16) unsigned char smem[];
  double* A = reinterpret_cast<double*>(smem);  // [epb][N3]
  double* Bb = A + epb * N3;                    // [epb][N3]
  double* red = Bb + epb * N3;                  // [epb][2][N3]
  const OpsTab<double>& O = ops<double>();
  const int tid = threadIdx.x, le = tid / N3, k = tid - le * N3;
  const int slot = blockIdx.x * epb + le;
  const bool act = le < epb && slot < nel;
  const int e = act ? elems[slot] : 0;
  const int i0 = k % N, i1 = (k / N) % N, i2 = k / N2;
  double s = 0.0;
  if (act) {
    s = U[(long)var * nsp + sp_off[e] + k];
    A[le * N3 + k] = s;
  }
  double* a = A + le * N3;
  double* b = Bb + le * N3;
  // nodal -> modal, one direction at a time (A -> B -> A -> B)
  __syncthreads();
  double t = 0.0;
  if (act)
    for (int m = 0; m < N; ++m) t += O.Vinv[N][i0][m] * a[m + N * (i1 + N * i2)];
  if (act) b[k] = t;
  __syncthreads();
  t = 0.0;
  if (act)
    for (int m = 0; m < N; ++m) t += O.Vinv[N][i1][m] * b[i0 + N * (m + N * i2)];
  __syncthreads();
  if (act) a[k] = t;
  __syncthreads();
  t = 0.0;
  if (act)
    for (int m = 0; m < N; ++m) t += O.Vinv[N][i2][m] * a[i0 + N * (i1 + N * m)];
  // keep the modes with some index equal to p
  if (act) b[k] = (i0 == N - 1 || i1 == N - 1 || i2 == N - 1) ? t : 0.0;
  __syncthreads();
  // modal -> nodal (B -> A -> B -> A)
  t = 0.0;
  if (act)
    for (int m = 0; m < N; ++m) t += O.V[N][i0][m] * b[m + N * (i1 + N * i2)];
  if (act) a[k] = t;
  __syncthreads();
  t = 0.0;
  if (act)
    for (int m = 0; m < N; ++m) t += O.V[N][i1][m] * a[i0 + N * (m + N * i2)];
  __syncthreads();
  if (act) b[k] = t;
  __syncthreads();
  t = 0.0;
  if (act)
    for (int m = 0; m < N; ++m) t += O.V[N][i2][m] * b[i0 + N * (i1 + N * m)];
  if (act) {
    double Ja[3][3], J;
    tri_metrics<double>(geo + 24L * e, O.x[N][i0], O.x[N][i1], O.x[N][i2], Ja, J);
    const double wJ = O.w[N][i0] * O.w[N][i1] * O.w[N][i2] * fabs(J);
    red[(le * 2 + 0) * N3 + k] = t * t * wJ;
    red[(le * 2 + 1) * N3 + k] = s * s * wJ;
  }
  __syncthreads();
  if (act && k == 0) {
    double num = 0.0, den = 0.0;
    for (int i = 0; i < N3; ++i) {
      num += red[(le * 2 + 0) * N3 + i];
      den += red[(le * 2 + 1) * N3 + i];
    }
    eta[e] = den > 0.0 ? num / den : 0.0;
  }
}

// eta_max = max_e eta_e (one block, fixed order)
__global__ void __launch_bounds__(256) k_max(const double* __restrict__ x, int n, double* __restrict__ out) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, x[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

}  // namespace frx
