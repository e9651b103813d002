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
// Factorisation: blocked LU with partial pivoting, one 256-thread block per
// element, the matrix column-major in device memory, then the inverse from
// the factors in place (the block is inverted through its LU, as the paper
// does).  Apply: the permutation and a dense product per element, in place.
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
// Entries reserved per block of order N: N^2 rounded up to 32, so that every
// block starts on a 128-byte boundary (float32 storage).
__host__ __device__ inline long pc_block_size(int N) { return ((long)N * N + 31) & ~31L; }
// Column stride of the float16 copy of a block (k_pc_to_half): N rounded up to
// 8, so that every column starts on a 16-byte boundary.
__host__ __device__ inline int pc_ld_half(int N) { return (N + 7) & ~7; }
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
// P A = L U with unit lower L; on return piv[i] = the row of A that is row i
// of P A (during the factorisation it holds the row swapped with row k at step k).
// Blocked, right-looking, one 256-thread block per element: a panel of PB
// columns (rows k0..N-1) is factored in LDS (pivot search, row swaps within
// the panel, scaling and the panel's own updates), written back, its swaps
// applied to the other columns, the panel's rows of the trailing columns
// solved with its unit lower triangle, and the trailing matrix updated once
// per panel (each thread holds the panel's multipliers of its rows in
// registers, U12 staged in LDS).  A zero pivot column (a singular block)
// sets *flag.  Launched per degree bucket (pc_lu_launch): ids lists the
// bucket's elements (null: element = block index), R (rows per thread,
// 256 R >= N), the panel width PB and the columns per trailing step CG are
// chosen by the block order, and the dynamic LDS holds PB N scalars.
constexpr int PC_NMAX = 5 * 6 * 6 * 6;            // largest block order (p = 5)
constexpr int PC_ROWS = (PC_NMAX + 255) / 256;    // rows per thread for every order
template <class TB> struct PcPanel { static constexpr int value = sizeof(TB) == 8 ? 8 : 16; };

template <class TB, int R, int PB, int CG>
__global__ void __launch_bounds__(256) k_pc_lu(TB* __restrict__ blocks, PcDev pc, const int* __restrict__ ids,
                                              int* __restrict__ piv, int* __restrict__ flag) {
  extern __shared__ __align__(16) unsigned char pc_lds[];
  TB* pan = reinterpret_cast<TB*>(pc_lds);  // [PB N]: pan[c * nr + (r - k0)], panel column c, rows k0..N-1
  __shared__ double red_v[4];  // one per wave of the 256-thread block
  __shared__ int red_i[4];
  __shared__ int pv[PB];
  __shared__ int mv_dst[2 * PB], mv_src[2 * PB], mv_cnt;
  const int el = ids ? ids[blockIdx.x] : (int)blockIdx.x;
  const int4 rec = pc.recs[el];
  const int N = pc_rows(rec.z);
  TB* A = blocks + pc.boff[el];
  int* P = piv + pc.poff[el];
  const int tid = threadIdx.x;
  for (int k0 = 0; k0 < N; k0 += PB) {
    const int w = min(PB, N - k0), nr = N - k0;
    // 1. the panel into LDS
    for (int t = tid; t < w * nr; t += blockDim.x) {
      const int c = t / nr, r = t - c * nr;
      pan[c * nr + r] = A[(k0 + r) + (long)(k0 + c) * N];
    }
    __syncthreads();
    // 2. unblocked LU of the panel
    for (int c = 0; c < w; ++c) {
      double best = -1.0;
      int bi = c;
      for (int r = c + tid; r < nr; r += blockDim.x) {
        const double v = fabs((double)pan[c * nr + r]);
        if (v > best) {
          best = v;
          bi = r;
        }
      }
      // the largest |value|, the lowest row among equal ones: within each
      // wave by shuffles, then over the waves' results in LDS
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o);
        const int oi = __shfl_xor(bi, o);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if ((tid & 63) == 0) {
        red_v[tid >> 6] = best;
        red_i[tid >> 6] = bi;
      }
      __syncthreads();
      best = red_v[0];
      bi = red_i[0];
      for (int wv = 1; wv < (int)(blockDim.x >> 6); ++wv) {
        const double ob = red_v[wv];
        const int oi = red_i[wv];
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      const int p = bi;
      const bool singular = !(best > 0.0);
      if (tid == 0) {
        pv[c] = p;
        P[k0 + c] = k0 + p;
        if (singular) *flag = 1;
      }
      if (p != c && tid < w) {
        const TB t = pan[tid * nr + c];
        pan[tid * nr + c] = pan[tid * nr + p];
        pan[tid * nr + p] = t;
      }
      __syncthreads();
      const TB inv = singular ? TB(0) : TB(1) / pan[c * nr + c];
      for (int r = c + 1 + tid; r < nr; r += blockDim.x) {
        const TB l = pan[c * nr + r] * inv;
        pan[c * nr + r] = l;
        for (int cc = c + 1; cc < w; ++cc) pan[cc * nr + r] -= l * pan[cc * nr + c];
      }
      __syncthreads();
    }
    // 3. the panel back
    for (int t = tid; t < w * nr; t += blockDim.x) {
      const int c = t / nr, r = t - c * nr;
      A[(k0 + r) + (long)(k0 + c) * N] = pan[c * nr + r];
    }
    // 4. the panel's row swaps on the other columns.  Their product is a
    // permutation of at most 2 w rows: replayed once on the row indices
    // (mv_dst[i] receives the old row mv_src[i], panel-relative), it moves
    // each column's rows with independent loads and then stores.
    if (tid == 0) {
      int cnt = 0;
      for (int c = 0; c < w; ++c) {
        const int p = pv[c];
        if (p == c) continue;
        int ic = -1, ip = -1;
        for (int i = 0; i < cnt; ++i) {
          if (mv_dst[i] == c) ic = i;
          if (mv_dst[i] == p) ip = i;
        }
        if (ic < 0) {
          ic = cnt++;
          mv_dst[ic] = mv_src[ic] = c;
        }
        if (ip < 0) {
          ip = cnt++;
          mv_dst[ip] = mv_src[ip] = p;
        }
        const int t = mv_src[ic];
        mv_src[ic] = mv_src[ip];
        mv_src[ip] = t;
      }
      mv_cnt = cnt;
    }
    __syncthreads();
    {
      const int cnt = mv_cnt;
      for (int j = tid; j < N; j += blockDim.x) {
        if (j >= k0 && j < k0 + w) continue;
        TB* col = A + k0 + (long)j * N;
        TB mv[2 * PB];
#pragma unroll
        for (int i = 0; i < 2 * PB; ++i)
          if (i < cnt) mv[i] = col[mv_src[i]];
#pragma unroll
        for (int i = 0; i < 2 * PB; ++i)
          if (i < cnt && mv_src[i] != mv_dst[i]) col[mv_dst[i]] = mv[i];
      }
    }
    __syncthreads();
    if (k0 + w >= N) break;
    // 5. the panel's rows of the trailing columns: solve with its unit lower triangle
    for (int j = k0 + w + tid; j < N; j += blockDim.x) {
      TB u[PB];
#pragma unroll
      for (int r = 0; r < PB; ++r) u[r] = r < w ? A[(k0 + r) + (long)j * N] : TB(0);
#pragma unroll
      for (int r = 1; r < PB; ++r)
#pragma unroll
        for (int t = 0; t < PB; ++t)
          if (t < r && r < w) u[r] -= pan[t * nr + r] * u[t];
#pragma unroll
      for (int r = 0; r < PB; ++r)
        if (r < w) A[(k0 + r) + (long)j * N] = u[r];
    }
    __syncthreads();
    // 6. trailing update A22 -= L21 U12, a thread per row (multipliers in registers)
    TB l[R][PB];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int r = w + tid + q * (int)blockDim.x;
#pragma unroll
      for (int t = 0; t < PB; ++t) l[q][t] = (r < nr && t < w) ? pan[t * nr + r] : TB(0);
    }
    __syncthreads();  // the panel is no longer read: U12 goes over it
    const int j0 = k0 + w, nt = N - j0;
    TB* u12 = pan;  // u12[(j - j0) PB + t] = U(k0 + t, j)
    for (int x = tid; x < nt * PB; x += blockDim.x) {
      const int jj = x / PB, t = x - jj * PB;
      u12[x] = t < w ? A[(k0 + t) + (long)(j0 + jj) * N] : TB(0);
    }
    __syncthreads();
    // CG columns per step: CG R independent loads per thread in flight
    for (int jj = 0; jj < nt; jj += CG) {
      TB a4[R][CG];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int r = w + tid + q * (int)blockDim.x;
#pragma unroll
        for (int c = 0; c < CG; ++c)
          a4[q][c] = (r < nr && jj + c < nt) ? A[(k0 + r) + (long)(j0 + jj + c) * N] : TB(0);
      }
#pragma unroll
      for (int c = 0; c < CG; ++c) {
        if (jj + c >= nt) break;
        TB u[PB];
#pragma unroll
        for (int t = 0; t < PB; ++t) u[t] = u12[(jj + c) * PB + t];
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
          for (int t = 0; t < PB; ++t) a4[q][c] -= l[q][t] * u[t];
      }
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int r = w + tid + q * (int)blockDim.x;
#pragma unroll
        for (int c = 0; c < CG; ++c)
          if (r < nr && jj + c < nt) A[(k0 + r) + (long)(j0 + jj + c) * N] = a4[q][c];
      }
    }
    __syncthreads();
  }
  // the swaps as one gather: perm[i] = the row of the original vector that
  // lands in row i after all of them (the swaps replayed on the identity,
  // serially, in LDS), stored over the swap list
  __syncthreads();
  static_assert(PB * sizeof(TB) >= 2 * sizeof(int), "the panel buffer holds the permutation");
  int* perm = reinterpret_cast<int*>(pan);
  int* sw = perm + N;
  for (int i = tid; i < N; i += blockDim.x) {
    perm[i] = i;
    sw[i] = P[i];
  }
  __syncthreads();
  if (tid == 0)
    for (int k = 0; k < N; ++k) {
      const int p = sw[k];
      if (p != k) {
        const int t = perm[k];
        perm[k] = perm[p];
        perm[p] = t;
      }
    }
  __syncthreads();
  for (int i = tid; i < N; i += blockDim.x) P[i] = perm[i];
}

// The LU of `count` blocks of order N (one degree bucket): rows per thread as
// few as the order allows, which leaves the registers for a wider panel (the
// trailing matrix is read and written once per panel: 24 float32 or 12
// float64 columns against 16 or 8, an 8 % shorter build at 128x128x8, where
// 32 float32 columns, with 2 trailing columns per step to stay in registers,
// gained less); blocks of order 1080 (p = 5) keep 5 rows and a narrow panel.
template <class TB, int R, int PB, int CG>
hipError_t pc_lu_shape(TB* blocks, const PcDev& pc, const int* ids, int count, int N, int* piv, int* flag,
                       hipStream_t s) {
  hipLaunchKernelGGL((k_pc_lu<TB, R, PB, CG>), dim3(count), dim3(256), (size_t)PB * N * sizeof(TB), s, blocks, pc,
                     ids, piv, flag);
  return hipGetLastError();
}
template <class TB>
hipError_t pc_lu_launch(TB* blocks, const PcDev& pc, const int* ids, int count, int N, int* piv, int* flag,
                        hipStream_t s) {
  constexpr int PB = sizeof(TB) == 8 ? 12 : 24;  // about 60 KB of LDS per block at N = 625
  if (N <= 256) return pc_lu_shape<TB, 1, PB, 4>(blocks, pc, ids, count, N, piv, flag, s);
  if (N <= 512) return pc_lu_shape<TB, 2, PB, 4>(blocks, pc, ids, count, N, piv, flag, s);
  if (N <= 768) return pc_lu_shape<TB, 3, PB, 4>(blocks, pc, ids, count, N, piv, flag, s);
  return pc_lu_shape<TB, PC_ROWS, PcPanel<TB>::value, 4>(blocks, pc, ids, count, N, piv, flag, s);
}

// The inverse of every factored block, in place: from the L\U of P A left
// by k_pc_lu, first U <- U^{-1} (column blocks of PB from the left: the
// block's rows above the diagonal are multiplied by the already inverted
// leading triangle and by minus the inverse of the block's own diagonal
// triangle, which is then inverted), then X L = U^{-1} is solved for X =
// (P A)^{-1} (column blocks from the right: the block's part of L is moved to
// LDS and cleared, the columns to its right are subtracted through it, and the
// block is solved with its unit lower triangle).  The block then holds
// (P A)^{-1}, so that A^{-1} x = (P A)^{-1} (P x): the apply gathers x
// through the permutation left in piv and multiplies.  One 256-thread block
// per element; a thread owns the R rows tid + 256 q (256 R >= N) and holds PB
// partial sums of each in registers, all R rows in one pass over the column
// index, so that one LDS value serves R rows and R loads are in flight per step;
// every loop over a column index reads a whole column (coalesced) per step.
// Launched per degree bucket (pc_inv_launch: ids, R by the block order, PB N
// scalars of dynamic LDS).
template <class TB, int R>
__global__ void __launch_bounds__(256) k_pc_inv(TB* __restrict__ blocks, PcDev pc, const int* __restrict__ ids) {
  constexpr int PB = PcPanel<TB>::value;
  extern __shared__ __align__(16) unsigned char pc_lds[];
  TB* wk = reinterpret_cast<TB*>(pc_lds);  // [PB N] the column block (above the diagonal, or its part of L), wk[row * PB + c]
  __shared__ TB dg[PB * PB];               // diagonal triangle of the column block, dg[c * PB + r]
  const int el = ids ? ids[blockIdx.x] : (int)blockIdx.x;
  const int4 rec = pc.recs[el];
  const int N = pc_rows(rec.z);
  TB* A = blocks + pc.boff[el];
  const int tid = threadIdx.x;
  const int base = tid & ~63;  // first row of this wave
  // 1. U <- U^{-1}
  for (int j0 = 0; j0 < N; j0 += PB) {
    const int jb = min(PB, N - j0);
    for (int t = tid; t < PB * j0; t += blockDim.x) {
      const int c = t / j0, r = t - c * j0;
      wk[r * PB + c] = c < jb ? A[r + (long)(j0 + c) * N] : TB(0);
    }
    for (int t = tid; t < PB * PB; t += blockDim.x) {
      const int c = t / PB, r = t - c * PB;
      dg[t] = (r < jb && c < jb) ? A[(j0 + r) + (long)(j0 + c) * N] : TB(1);
    }
    __syncthreads();
    if (base < j0) {  // rows above the block in this wave (their rows i >= base)
      TB acc[R][PB];
#pragma unroll
      for (int q = 0; q < R; ++q)
#pragma unroll
        for (int c = 0; c < PB; ++c) acc[q][c] = TB(0);
#pragma unroll 4
      for (int k = base; k < j0; ++k) {  // (U^{-1})[i, k] for k >= i, times the old column block
        TB u[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = tid + q * (int)blockDim.x;
          u[q] = (i < j0 && k >= i) ? A[i + (long)k * N] : TB(0);
        }
        const TB* w = wk + k * PB;
#pragma unroll
        for (int c = 0; c < PB; ++c) {
          const TB wc = w[c];
#pragma unroll
          for (int q = 0; q < R; ++q) acc[q][c] += u[q] * wc;
        }
      }
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int i = tid + q * (int)blockDim.x;
        // X D = -acc with D the block's upper diagonal triangle
#pragma unroll
        for (int c = 0; c < PB; ++c) {
          TB v = -acc[q][c];
#pragma unroll
          for (int k = 0; k < PB; ++k)
            if (k < c) v -= acc[q][k] * dg[c * PB + k];
          acc[q][c] = v / dg[c * PB + c];
        }
        if (i < j0)
#pragma unroll
          for (int c = 0; c < PB; ++c)
            if (c < jb) A[i + (long)(j0 + c) * N] = acc[q][c];
      }
    }
    // the diagonal triangle's inverse, a row per thread
    if (tid < jb) {
      const int r = tid;
      TB row[PB];
#pragma unroll
      for (int c = 0; c < PB; ++c) {
        if (c < r || c >= jb) {
          row[c] = TB(0);
        } else if (c == r) {
          row[c] = TB(1) / dg[c * PB + c];
        } else {
          TB v = TB(0);
#pragma unroll
          for (int k = 0; k < PB; ++k)
            if (k >= r && k < c) v += row[k] * dg[c * PB + k];
          row[c] = -v / dg[c * PB + c];
        }
      }
#pragma unroll
      for (int c = 0; c < PB; ++c)
        if (c >= r && c < jb) A[(j0 + r) + (long)(j0 + c) * N] = row[c];
    }
    __syncthreads();
  }
  // 2. X L = U^{-1}, column blocks from the right
  for (int j0 = ((N - 1) / PB) * PB; j0 >= 0; j0 -= PB) {
    const int jb = min(PB, N - j0), nw = N - j0;
    for (int t = tid; t < PB * nw; t += blockDim.x) {
      const int c = t / nw, r = t - c * nw;
      TB* a = A + (j0 + r) + (long)(j0 + c) * N;
      if (r > c && c < jb) {
        wk[r * PB + c] = *a;
        *a = TB(0);
      } else {
        wk[r * PB + c] = TB(0);
      }
    }
    __syncthreads();
    if (base < N) {
      TB acc[R][PB];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int i = tid + q * (int)blockDim.x;
#pragma unroll
        for (int c = 0; c < PB; ++c) acc[q][c] = (i < N && c < jb) ? A[i + (long)(j0 + c) * N] : TB(0);
      }
#pragma unroll 4
      for (int k = j0 + jb; k < N; ++k) {
        TB x[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = tid + q * (int)blockDim.x;
          x[q] = i < N ? A[i + (long)k * N] : TB(0);
        }
        const TB* w = wk + (k - j0) * PB;
#pragma unroll
        for (int c = 0; c < PB; ++c) {
          const TB wc = w[c];
#pragma unroll
          for (int q = 0; q < R; ++q) acc[q][c] -= x[q] * wc;
        }
      }
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int i = tid + q * (int)blockDim.x;
        // X Ld = acc with Ld the unit lower triangle of the block's L part
#pragma unroll
        for (int c = PB - 1; c >= 0; --c) {
          TB v = acc[q][c];
#pragma unroll
          for (int k = 0; k < PB; ++k)
            if (k > c && k < jb) v -= acc[q][k] * wk[k * PB + c];
          acc[q][c] = v;
        }
        if (i < N)
#pragma unroll
          for (int c = 0; c < PB; ++c)
            if (c < jb) A[i + (long)(j0 + c) * N] = acc[q][c];
      }
    }
    __syncthreads();
  }
}

// The inverse of `count` factored blocks of order N (one degree bucket): rows
// per thread as few as the order allows.
template <class TB>
hipError_t pc_inv_launch(TB* blocks, const PcDev& pc, const int* ids, int count, int N, hipStream_t s) {
  const size_t lds = (size_t)PcPanel<TB>::value * N * sizeof(TB);
  if (N <= 256)
    hipLaunchKernelGGL((k_pc_inv<TB, 1>), dim3(count), dim3(256), lds, s, blocks, pc, ids);
  else if (N <= 512)
    hipLaunchKernelGGL((k_pc_inv<TB, 2>), dim3(count), dim3(256), lds, s, blocks, pc, ids);
  else if (N <= 768)
    hipLaunchKernelGGL((k_pc_inv<TB, 3>), dim3(count), dim3(256), lds, s, blocks, pc, ids);
  else
    hipLaunchKernelGGL((k_pc_inv<TB, PC_ROWS>), dim3(count), dim3(256), lds, s, blocks, pc, ids);
  return hipGetLastError();
}

// x_e <- A_e^{-1} x_e from the float16 copy of sigma (P A)^{-1} that
// k_pc_to_half leaves: z = P x (float, LDS), the product accumulated in
// float32 and scaled by sc = 1/sigma.  Called by k_pc_apply (float32
// storage) when the device flag asks for it; shapes as there.
// The float16 copy has column stride pc_ld_half(N): a thread owns 8
// consecutive rows and reads them with one 16-byte load per column; the
// columns are split over blockDim.x / (LD / 8) groups of threads, whose
// partial sums meet in LDS (part: at least 8 blockDim.x floats).
template <class TV>
__device__ void pc_apply_half(TV* __restrict__ x, int nsp, const float* __restrict__ blocks, const PcDev& pc,
                              const int* __restrict__ piv, float sc, float* z, float* part) {
  const int4 r = pc.recs[blockIdx.x];
  const int N = pc_rows(r.z), LD = pc_ld_half(N);
  const _Float16* A = reinterpret_cast<const _Float16*>(blocks + pc.boff[blockIdx.x]);
  const int* P = piv + pc.poff[blockIdx.x];
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += blockDim.x) z[i] = (float)x[pc_dof(P[i], r.z, r.y, nsp)];
  __syncthreads();
  const int nrg = LD / 8;                           // row groups, at most PC_NMAX / 8 = 135
  const int ncg = (int)blockDim.x / nrg;            // column groups, at least 1
  const int rg = tid % nrg, cg = tid / nrg;
  if (cg < ncg) {
    float acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0f;
    const int k0 = cg * N / ncg, k1 = (cg + 1) * N / ncg;
    const _Float16* col = A + 8 * rg;
#pragma unroll 4
    for (int k = k0; k < k1; ++k) {
      const uint4 w = *reinterpret_cast<const uint4*>(col + (long)k * LD);
      const _Float16* h = reinterpret_cast<const _Float16*>(&w);
      const float zk = z[k];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] += (float)h[q] * zk;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) part[cg * LD + 8 * rg + q] = acc[q];
  }
  __syncthreads();
  for (int i = tid; i < N; i += blockDim.x) {
    float s = 0.0f;
    for (int g = 0; g < ncg; ++g) s += part[g * LD + i];
    x[pc_dof(i, r.z, r.y, nsp)] = (TV)(s * sc);
  }
}

// x_e <- A_e^{-1} x_e for every element, in place (x: the Krylov vector, TV
// storage; the product runs in TB): x is gathered through the permutation
// (z = P x, in LDS), then multiplied by the stored (P A)^{-1}.  Rows over the
// threads; blocks of at most 128 rows split the columns over 2 or 4 groups of
// threads and add the partial sums in LDS.  The device flag *on selects: 0
// leaves x unchanged, 1 the stored inverse, 2 (float32 storage) its float16
// copy with *isig = 1/sigma; so one captured graph serves the plain and both
// preconditioned solves, whichever was built last.  *done != 0 returns at
// once, as every kernel of a captured Arnoldi step.
template <class TV, class TB>
__global__ void __launch_bounds__(256) k_pc_apply(TV* __restrict__ x, int nsp, const TB* __restrict__ blocks, PcDev pc,
                                                 const int* __restrict__ piv, const int* __restrict__ on,
                                                 const int* __restrict__ done, const double* __restrict__ isig) {
  const int mode = *on;
  if (!mode || (done && *done)) return;
  __shared__ TB z[PC_NMAX];
  __shared__ TB part[sizeof(TB) == 4 ? 8 * 256 : 256];  // float32 storage: also the float16 path's partial sums
  if constexpr (sizeof(TB) == 4) {
    if (mode == 2) {
      pc_apply_half<TV>(x, nsp, (const float*)blocks, pc, piv, (float)*isig, (float*)z, (float*)part);
      return;
    }
  }
  const int4 r = pc.recs[blockIdx.x];
  const int N = pc_rows(r.z);
  const TB* A = blocks + pc.boff[blockIdx.x];
  const int* P = piv + pc.poff[blockIdx.x];
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += blockDim.x) z[i] = (TB)x[pc_dof(P[i], r.z, r.y, nsp)];
  __syncthreads();
  const int slots = (N + 63) & ~63;  // rows padded to whole waves
  if (slots <= 128) {
    const int groups = 256 / slots, g = tid / slots, i = tid - g * slots;
    const int k0 = g * N / groups, k1 = (g + 1) * N / groups;
    TB acc = TB(0);
    if (i < N)
      for (int k = k0; k < k1; ++k) acc += A[i + (long)k * N] * z[k];
    part[tid] = acc;
    __syncthreads();
    if (g == 0 && i < N) {
      for (int h = 1; h < groups; ++h) acc += part[h * slots + i];
      x[pc_dof(i, r.z, r.y, nsp)] = (TV)acc;
    }
    return;
  }
  for (int i0 = tid & ~63; i0 < N; i0 += blockDim.x) {
    const int i = i0 + (tid & 63);
    if (i >= N) break;
    TB a0 = TB(0), a1 = TB(0), a2 = TB(0), a3 = TB(0);
    int k = 0;
    for (; k + 4 <= N; k += 4) {
      a0 += A[i + (long)k * N] * z[k];
      a1 += A[i + (long)(k + 1) * N] * z[k + 1];
      a2 += A[i + (long)(k + 2) * N] * z[k + 2];
      a3 += A[i + (long)(k + 3) * N] * z[k + 3];
    }
    for (; k < N; ++k) a0 += A[i + (long)k * N] * z[k];
    x[pc_dof(i, r.z, r.y, nsp)] = (TV)((a0 + a1) + (a2 + a3));
  }
}

// Half-precision copy of the inverse for the apply (float32 build): every
// element's float32 (P A)^{-1} is replaced, in place at the start of its own
// block, by float16 values of sigma (P A)^{-1} (entries of order one, since
// the blocks are sigma I minus the Jacobian block), column-major with column
// stride LD = pc_ld_half(N) and zero pad rows.  A chunk of 256 entries is
// read, then written after a barrier: float32 entry k = c N + r ends at byte
// 4 (k + 1), its float16 value (and, for r = N - 1, the pad of column c) ends
// at byte 2 (c LD + r + 1) <= 4 (k + 1) (or 2 (c + 1) LD <= 4 (k + 1)), as
// LD <= 2 N: a chunk's float16 values cover float32 entries of the same or
// earlier chunks only.  One 256-thread block per element (blockDim.x = 256),
// per degree bucket (ids).
__global__ void __launch_bounds__(256) k_pc_to_half(float* __restrict__ blocks, PcDev pc, const int* __restrict__ ids,
                                                   double sigma) {
  const int el = ids ? ids[blockIdx.x] : (int)blockIdx.x;
  const int N = pc_rows(pc.recs[el].z);
  float* A = blocks + pc.boff[el];
  _Float16* H = reinterpret_cast<_Float16*>(A);
  const long NN = (long)N * N;
  const int LD = pc_ld_half(N);
  const float sg = (float)sigma;
  __shared__ float stage[256];
  for (long k0 = 0; k0 < NN; k0 += blockDim.x) {
    const long k = k0 + threadIdx.x;
    // through LDS, so that every load of the chunk has returned (its value
    // stored in LDS) before the barrier that precedes the overwriting stores
    stage[threadIdx.x] = k < NN ? A[k] : 0.0f;
    __syncthreads();
    if (k < NN) {
      const int c = (int)(k / N), r = (int)(k - (long)c * N);
      H[(long)c * LD + r] = (_Float16)(sg * stage[threadIdx.x]);
      if (r == N - 1)
        for (int q = N; q < LD; ++q) H[(long)c * LD + q] = (_Float16)0.0f;
    }
    __syncthreads();
  }
}

}  // namespace frx
