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

// out[n] = max of eta_e over the elements of size n = p + 1 (n = 2..6; 0 where
// there is none), one block, fixed order
__global__ void __launch_bounds__(256) k_max_by_degree(const double* __restrict__ x, const int8_t* __restrict__ p,
                                                      int n, double* __restrict__ out) {
  __shared__ double sh[NMAX + 1][256];
  double m[NMAX + 1];
#pragma unroll
  for (int k = 0; k <= NMAX; ++k) m[k] = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const int k = p[i] + 1;
#pragma unroll
    for (int j = 2; j <= NMAX; ++j)
      if (k == j) m[j] = fmax(m[j], x[i]);
  }
#pragma unroll
  for (int k = 0; k <= NMAX; ++k) sh[k][threadIdx.x] = m[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
#pragma unroll
      for (int k = 0; k <= NMAX; ++k) sh[k][threadIdx.x] = fmax(sh[k][threadIdx.x], sh[k][threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x <= NMAX) out[threadIdx.x] = sh[threadIdx.x][0];
}

}  // namespace frx

namespace frx {

// ------------------------------------------------------- degree selection
// Criteria of section 3.1 from the indicator: raise p by one where
// eta > nu_max eta_max, lower it by one where eta < nu_min eta_max, clamped to
// [p_min, p_max] (decided in float64).  eta_max is the maximum over all
// elements (by_degree = 0: eta_max[0]) or over the elements of the same degree
// (by_degree = 1: eta_max[p + 1]).  One thread per element.
__global__ void __launch_bounds__(256) k_select(const double* __restrict__ eta, const double* __restrict__ eta_max,
                                               int by_degree, const int8_t* __restrict__ p, int E, double nu_max,
                                               double nu_min, int p_min, int p_max, int8_t* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const double m = by_degree ? eta_max[p[e] + 1] : eta_max[0];
  int q = p[e] + (eta[e] > nu_max * m ? 1 : 0) - (eta[e] < nu_min * m ? 1 : 0);
  q = q < p_min ? p_min : (q > p_max ? p_max : q);
  out[e] = (int8_t)q;
}

// One sweep of the face limiter: the lower side of a face whose degrees
// differ by more than one is raised, out[e] = max(in[e], max_nb in[nb] - 1).
// p_max - p_min sweeps reach the fixed point (a degree constraint travels one
// element per sweep and loses one degree per element).
__global__ void __launch_bounds__(256) k_limit(const int8_t* __restrict__ in, const int* __restrict__ nbr, int E,
                                              int8_t* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  int q = in[e];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int nb = nbr[6 * e + f];
    if (nb >= 0) q = max(q, (int)in[nb] - 1);
  }
  out[e] = (int8_t)q;
}

// Projection of a state between two degree fields of the same mesh, one block
// per element: the element polynomial through its ns^3 Gauss points is
// expanded in Legendre modes (Vinv), truncated to the modes below nd in every
// direction and evaluated at the nd^3 Gauss points (V):
//   M[i][a] = sum_{m < min(ns, nd)} P_m(x^nd_i) (2m+1)/2 w^ns_a P_m(x^ns_a),
// applied in the three directions (the reference-space L2 projection when
// nd < ns, exact interpolation otherwise).
__global__ void __launch_bounds__(256) k_project(const double* __restrict__ Us, int nsp_s, const int* __restrict__ off_s,
                                                const int8_t* __restrict__ p_s, double* __restrict__ Ud, int nsp_d,
                                                const int* __restrict__ off_d, const int8_t* __restrict__ p_d) {
  __shared__ double M[NMAX][NMAX];
  __shared__ double u[5][NMAX * NMAX * NMAX];
  const OpsTab<double>& O = ops<double>();
  const int e = blockIdx.x;
  const int ns = p_s[e] + 1, nd = p_d[e] + 1, ns3 = ns * ns * ns, nd3 = nd * nd * nd;
  const int mm = min(ns, nd);
  const int t = threadIdx.x;
  if (t < nd * ns) {
    const int i = t / ns, a = t - i * ns;
    double s = 0.0;
    for (int m = 0; m < mm; ++m) s += O.V[nd][i][m] * O.Vinv[ns][m][a];
    M[i][a] = s;
  }
  for (int k = t; k < 5 * ns3; k += blockDim.x) {
    const int v = k / ns3, q = k - v * ns3;
    u[v][q] = Us[(long)v * nsp_s + off_s[e] + q];
  }
  __syncthreads();
  if (t >= nd3) return;
  const int i0 = t % nd, i1 = (t / nd) % nd, i2 = t / (nd * nd);
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int c = 0; c < ns; ++c)
    for (int b = 0; b < ns; ++b) {
      const double mbc = M[i2][c] * M[i1][b];
      for (int a = 0; a < ns; ++a) {
        const double w = mbc * M[i0][a];
        const int q = a + ns * (b + ns * c);
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v] += w * u[v][q];
      }
    }
#pragma unroll
  for (int v = 0; v < 5; ++v) Ud[(long)v * nsp_d + off_d[e] + t] = acc[v];
}

// Nodal polynomial filter of the elements of size N (section 4.2, the
// SD7003 case; the filter of Fischer and Mullen): q <- (1 - alpha) q +
// alpha Pi q with Pi the reference-space L2 projection onto the tensor
// polynomials of degree N - 2, i.e. the highest Legendre mode of each
// direction removed, evaluated at the element's Gauss points.  One block per
// element (N^3 threads used); Pi is applied direction by direction with the
// N x N matrix M[i][a] = sum_{m < N-1} P_m(x_i) (2m+1)/2 w_a P_m(x_a).
// Uout may be U: a block reads its element completely before writing it.
template <int N>
__global__ void __launch_bounds__(256) k_filter(const double* U, int nsp, const int4* __restrict__ recs,
                                               double alpha, double* Uout) {
  constexpr int N3 = N * N * N;
  __shared__ double M[N][N];
  __shared__ double X[5][N3], Y[5][N3];
  const OpsTab<double>& O = ops<double>();
  const int t = threadIdx.x;
  const long off = recs[blockIdx.x].y;
  if (t < N * N) {
    const int i = t / N, a = t - i * N;
    double s = 0.0;
    for (int m = 0; m < N - 1; ++m) s += O.V[N][i][m] * O.Vinv[N][m][a];
    M[i][a] = s;
  }
  double q[5];
  if (t < N3) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      q[v] = U[(long)v * nsp + off + t];
      X[v][t] = q[v];
    }
  }
  const int i0 = t % N, i1 = (t / N) % N, i2 = t / (N * N);
  __syncthreads();
  if (t < N3) {  // along xi
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < N; ++a) s += M[i0][a] * X[v][a + N * (i1 + N * i2)];
      Y[v][t] = s;
    }
  }
  __syncthreads();
  if (t < N3) {  // along eta
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < N; ++b) s += M[i1][b] * Y[v][i0 + N * (b + N * i2)];
      X[v][t] = s;
    }
  }
  __syncthreads();
  if (t < N3) {  // along zeta, then the blend
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < N; ++c) s += M[i2][c] * X[v][i0 + N * (i1 + N * c)];
      Uout[(long)v * nsp + off + t] = (1.0 - alpha) * q[v] + alpha * s;
    }
  }
}

}  // namespace frx
