// Exchange operator in adaptively compressed form (Sec. IV: the exchange
// enters the self-consistent iteration through the compressed operator of
// Lin, J. Chem. Theory Comput. 12, 2242 (2016)).  From W = Vx psi:
//   M = (psi_j, W_k)_h,  -M = L L^T,  xi = L^{-1} W,
//   V_ACE phi = -sum_k xi_k (xi_k, phi)_h.
// The fields are long rows (norb x N, N up to millions) and the coupling
// matrices small (norb x norb), so the work is three memory-bound shapes:
//   gram     C = A B^T over the grid points (split over point ranges into
//            partial sums, then reduced in a fixed order: bitwise repeatable);
//   chol_inv the Cholesky factor of the small matrix and its inverse, one
//            workgroup;
//   combine  Out = alpha C X (each output row a combination of the rows of X),
//            one pass over X and Out.
// FP64 arithmetic throughout; fields stored as double or float.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kx_internal.h"

namespace kx {
namespace {

constexpr int kGT = 128;      // gram: rows of A and of B per workgroup tile
constexpr int kGK = 16;       // gram: grid points per staged step
constexpr int kGLd = kGT + 2; // LDS row stride of the staged tiles (doubles)
constexpr int kCV = 128;      // combine: output rows per workgroup
constexpr int kCR = 64;       // combine: grid points per workgroup
constexpr int kCK = 16;       // combine: rows of X per staged step

// part[grp][i][j] = sum over points r of group grp of A[i][r] B[j][r].
// 256 threads as a 16 x 16 grid, each owning an 8 x 8 block of the tile.
template <class SA, class SB>
__global__ void __launch_bounds__(256) gram_partial(const SA* __restrict__ A, int na,
                                                    const SB* __restrict__ B, int nb, long long N,
                                                    long long per, double* __restrict__ part) {
  __shared__ double As[kGK * kGLd];
  __shared__ double Bs[kGK * kGLd];
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  const int i0 = blockIdx.y * kGT, j0 = blockIdx.z * kGT;
  const long long r0 = (long long)blockIdx.x * per;
  const long long r1 = r0 + per < N ? r0 + per : N;
  // staging: thread t loads 8 consecutive points of row t / 2 of each tile
  const int lrow = t >> 1, lcol = (t & 1) * 8;
  const bool ain = i0 + lrow < na, bin = j0 + lrow < nb;
  const SA* __restrict__ arow = A + (long long)(ain ? i0 + lrow : 0) * N;
  const SB* __restrict__ brow = B + (long long)(bin ? j0 + lrow : 0) * N;
  double acc[8][8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[a][b] = 0.0;
  // the next step's values are loaded into registers while this step is
  // multiplied
  double na_[8], nb_[8];
  auto fetch = [&](long long rb) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const long long r = rb + lcol + c;
      const bool rin = r < r1;
      na_[c] = (ain && rin) ? (double)arow[r] : 0.0;
      nb_[c] = (bin && rin) ? (double)brow[r] : 0.0;
    }
  };
  if (r0 < r1) fetch(r0);
  for (long long rb = r0; rb < r1; rb += kGK) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      As[(lcol + c) * kGLd + lrow] = na_[c];
      Bs[(lcol + c) * kGLd + lrow] = nb_[c];
    }
    __syncthreads();
    if (rb + kGK < r1) fetch(rb + kGK);
#pragma unroll 4
    for (int k = 0; k < kGK; ++k) {
      double av[8], bv[8];
#pragma unroll
      for (int a = 0; a < 8; ++a) av[a] = As[k * kGLd + ty * 8 + a];
#pragma unroll
      for (int b = 0; b < 8; ++b) bv[b] = Bs[k * kGLd + tx * 8 + b];
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  double* __restrict__ pg = part + (long long)blockIdx.x * na * nb;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int i = i0 + ty * 8 + a;
    if (i >= na) continue;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int j = j0 + tx * 8 + b;
      if (j < nb) pg[(long long)i * nb + j] = acc[a][b];
    }
  }
}

// out[i][j] = scale * sum_grp part[grp][i][j], groups in index order
__global__ void __launch_bounds__(256) gram_reduce(const double* __restrict__ part, int ngrp,
                                                   long long nn, double scale,
                                                   double* __restrict__ out) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nn) return;
  double s = 0.0;
  for (int grp = 0; grp < ngrp; ++grp) s += part[(long long)grp * nn + k];
  out[k] = scale * s;
}

// A (n x n, symmetric, lower triangle used) is overwritten by its Cholesky
// factor L (A = L L^T, right-looking, one workgroup); then Linv = L^{-1}
// (lower triangular, upper part zero), one column per thread by forward
// substitution.  status = 0, or k + 1 when the k-th pivot is not positive
// (A is not positive definite); Linv is not written then.
__global__ void __launch_bounds__(1024) chol_inv(double* __restrict__ A, int n,
                                                 double* __restrict__ Linv, int* status) {
  const int t = threadIdx.x, nt = blockDim.x;
  const int tx = t & 31, ty = t >> 5, nx = 32, ny = nt >> 5;
  __shared__ int fail;
  if (t == 0) fail = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (t == 0) {
      const double d = A[(long long)k * n + k];
      if (d > 0.0 && std::isfinite(d))
        A[(long long)k * n + k] = sqrt(d);
      else
        fail = k + 1;
    }
    __syncthreads();
    if (fail) break;
    const double dk = A[(long long)k * n + k];
    for (int i = k + 1 + t; i < n; i += nt) A[(long long)i * n + k] /= dk;
    __syncthreads();
    for (int i = k + 1 + ty; i < n; i += ny) {
      const double lik = A[(long long)i * n + k];
      for (int j = k + 1 + tx; j <= i; j += nx)
        A[(long long)i * n + j] -= lik * A[(long long)j * n + k];
    }
    __syncthreads();
  }
  if (t == 0) *status = fail;
  if (fail) return;
  for (int c = t; c < n; c += nt) {
    for (int i = 0; i < c; ++i) Linv[(long long)i * n + c] = 0.0;
    Linv[(long long)c * n + c] = 1.0 / A[(long long)c * n + c];
    for (int i = c + 1; i < n; ++i) {
      double s = 0.0;
      for (int k = c; k < i; ++k) s += A[(long long)i * n + k] * Linv[(long long)k * n + c];
      Linv[(long long)i * n + c] = -s / A[(long long)i * n + i];
    }
  }
}

// Out[v][r] = alpha * sum_k C[v * ldv + k * ldk] X[k][r], v < m, k < n.
// 256 threads as 16 (points) x 16 (rows), each owning 8 rows x 4 points.
template <class S>
__global__ void __launch_bounds__(256) combine(const double* __restrict__ C, long long ldv,
                                               long long ldk, int m, int n,
                                               const S* __restrict__ X, long long N, double alpha,
                                               S* __restrict__ Out) {
  __shared__ double Xs[kCK * kCR];
  __shared__ double Cs[kCK * (kCV + 2)];
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  const long long r0 = (long long)blockIdx.x * kCR;
  const int v0 = blockIdx.y * kCV;
  double acc[8][4];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  // staging: X rows k0 + t / 16, points 4 (t % 16) ..; C rows v0 + t / 2,
  // columns k0 + 8 (t % 2) ..
  const int xk = t >> 4, xr = (t & 15) * 4;
  const int cv = t >> 1, ck = (t & 1) * 8;
  // the next step's values are loaded into registers while this step is
  // multiplied
  double nx[4], nc[8];
  auto fetch = [&](int k0) {
    const int k = k0 + xk;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const long long r = r0 + xr + b;
      nx[b] = (k < n && r < N) ? (double)X[(long long)k * N + r] : 0.0;
    }
    const int v = v0 + cv;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int k2 = k0 + ck + c;
      nc[c] = (v < m && k2 < n) ? C[v * ldv + k2 * ldk] : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < n; k0 += kCK) {
#pragma unroll
    for (int b = 0; b < 4; ++b) Xs[xk * kCR + xr + b] = nx[b];
#pragma unroll
    for (int c = 0; c < 8; ++c) Cs[(ck + c) * (kCV + 2) + cv] = nc[c];
    __syncthreads();
    if (k0 + kCK < n) fetch(k0 + kCK);
#pragma unroll 4
    for (int k = 0; k < kCK; ++k) {
      double cvv[8], xv[4];
#pragma unroll
      for (int a = 0; a < 8; ++a) cvv[a] = Cs[k * (kCV + 2) + ty * 8 + a];
#pragma unroll
      for (int b = 0; b < 4; ++b) xv[b] = Xs[k * kCR + tx * 4 + b];
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(cvv[a], xv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int v = v0 + ty * 8 + a;
    if (v >= m) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const long long r = r0 + tx * 4 + b;
      if (r < N) Out[(long long)v * N + r] = (S)(alpha * acc[a][b]);
    }
  }
}

}  // namespace

long long ace_groups(long long N, int na, int nb) {
  // about four workgroups per CU when the partial sums allow it
  long long grp = (N + 511) / 512;
  if (grp > 1024) grp = 1024;
  const long long cap = (128ll << 20) / ((long long)na * nb * (long long)sizeof(double));
  if (grp > cap) grp = cap;
  return grp < 1 ? 1 : grp;
}

hipError_t launch_gram(int storage, const void* A, int na, const void* B, int nb, long long N,
                       long long ngrp, double* part, double scale, double* out, hipStream_t s) {
  if (na <= 0 || nb <= 0 || N <= 0 || ngrp <= 0) return hipErrorInvalidValue;
  long long per = (N + ngrp - 1) / ngrp;
  per = (per + kGK - 1) / kGK * kGK;
  const long long used = (N + per - 1) / per;  // groups that hold points
  const dim3 grid((unsigned)used, (unsigned)((na + kGT - 1) / kGT), (unsigned)((nb + kGT - 1) / kGT));
  if (storage == KX_F64)
    hipLaunchKernelGGL((gram_partial<double, double>), grid, dim3(256), 0, s, (const double*)A, na,
                       (const double*)B, nb, N, per, part);
  else
    hipLaunchKernelGGL((gram_partial<float, float>), grid, dim3(256), 0, s, (const float*)A, na,
                       (const float*)B, nb, N, per, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long nn = (long long)na * nb;
  hipLaunchKernelGGL(gram_reduce, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, part,
                     (int)used, nn, scale, out);
  return hipGetLastError();
}

hipError_t launch_chol_inv(double* A, int n, double* Linv, int* status, hipStream_t s) {
  if (n <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(chol_inv, dim3(1), dim3(1024), 0, s, A, n, Linv, status);
  return hipGetLastError();
}

hipError_t launch_combine(int storage, const double* C, long long ldv, long long ldk, int m, int n,
                          const void* X, long long N, double alpha, void* Out, hipStream_t s) {
  if (m <= 0 || n <= 0 || N <= 0) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((N + kCR - 1) / kCR), (unsigned)((m + kCV - 1) / kCV));
  if (storage == KX_F64)
    hipLaunchKernelGGL((combine<double>), grid, dim3(256), 0, s, C, ldv, ldk, m, n,
                       (const double*)X, N, alpha, (double*)Out);
  else
    hipLaunchKernelGGL((combine<float>), grid, dim3(256), 0, s, C, ldv, ldk, m, n,
                       (const float*)X, N, alpha, (float*)Out);
  return hipGetLastError();
}

}  // namespace kx
