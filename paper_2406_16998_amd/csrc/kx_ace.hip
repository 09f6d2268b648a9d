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
// The gram and the combination are dense contractions on FP64 MFMA tiles
// (staging through LDS, next step prefetched into registers).  FP64
// arithmetic throughout; fields stored as double or float.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "kx_aux.h"
#include "kx_internal.h"

namespace kx {
namespace {

constexpr int kGT = 128;      // gram: rows of A and of B per workgroup tile
constexpr int kGK = 16;       // gram: grid points per staged step
constexpr int kGLd = kGT + 2; // LDS row stride of the staged tiles (doubles)
constexpr int kCV = 128;      // combine: output rows per workgroup
constexpr int kCR = 64;       // combine: grid points per workgroup
constexpr int kCK = 16;       // combine: rows of X per staged step

// eight consecutive values (16-byte aligned) widened to double
__device__ __forceinline__ void load8(const double* p, double* v) {
  typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const d2 x = *reinterpret_cast<const d2*>(p + 2 * q);
    v[2 * q] = x[0];
    v[2 * q + 1] = x[1];
  }
}
__device__ __forceinline__ void load8(const float* p, double* v) {
  typedef float f4 __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const f4 x = *reinterpret_cast<const f4*>(p + 4 * q);
#pragma unroll
    for (int e = 0; e < 4; ++e) v[4 * q + e] = (double)x[e];
  }
}

// four consecutive values (16-byte aligned) widened to double
__device__ __forceinline__ void load4(const double* p, double* v) {
  typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const d2 x = *reinterpret_cast<const d2*>(p + 2 * q);
    v[2 * q] = x[0];
    v[2 * q + 1] = x[1];
  }
}
__device__ __forceinline__ void load4(const float* p, double* v) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const f4 x = *reinterpret_cast<const f4*>(p);
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = (double)x[e];
}

// part[grp][i][j] = sum over points r of group grp of A[i][r] B[j][r].
// 256 threads = 4 waves; wave w owns the 64 x 64 quarter (w / 2, w % 2) of
// the 128 x 128 tile as 4 x 4 blocks of 16 x 16 on v_mfma_f64_16x16x4f64
// (lane l = 16 lg + li holds A[li][lg] and B[lg][li]; element e of a block
// accumulator holds D[4 e + lg][li]).  The staged points are the products'
// K dimension: A[m][k] = As[k][m], B[k][n] = Bs[k][n].
template <class SA, class SB>
__global__ void __launch_bounds__(256) gram_partial(const SA* __restrict__ A, int na,
                                                    const SB* __restrict__ B, int nb, long long N,
                                                    long long per, double* __restrict__ part) {
  typedef double v4d __attribute__((ext_vector_type(4)));
  __shared__ double As[kGK * kGLd];
  __shared__ double Bs[kGK * kGLd];
  const int t = threadIdx.x;
  const int lane = t & 63, li = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int wi = (wave >> 1) * 64, wj = (wave & 1) * 64;
  const int i0 = blockIdx.y * kGT, j0 = blockIdx.z * kGT;
  const long long r0 = (long long)blockIdx.x * per;
  const long long r1 = r0 + per < N ? r0 + per : N;
  // staging: thread t loads 8 consecutive points of row t / 2 of each tile
  const int lrow = t >> 1, lcol = (t & 1) * 8;
  const bool ain = i0 + lrow < na, bin = j0 + lrow < nb;
  const SA* __restrict__ arow = A + (long long)(ain ? i0 + lrow : 0) * N;
  const SB* __restrict__ brow = B + (long long)(bin ? j0 + lrow : 0) * N;
  v4d acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0, 0, 0, 0};
  // the next step's values are loaded into registers while this step is
  // multiplied
  double na_[8], nb_[8];
  // whole steps of rows that exist, on 16-byte aligned rows: 16-byte loads
  const bool vec = ((N * (long long)sizeof(SA)) % 16 == 0) && ((N * (long long)sizeof(SB)) % 16 == 0) &&
                   ((reinterpret_cast<unsigned long long>(A) | reinterpret_cast<unsigned long long>(B)) & 15) == 0;
  auto fetch = [&](long long rb) {
    if (vec && ain && bin && rb + kGK <= r1 && (rb & 7) == 0) {
      load8(arow + rb + lcol, na_);
      load8(brow + rb + lcol, nb_);
      return;
    }
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
#pragma unroll
    for (int k4 = 0; k4 < kGK; k4 += 4) {
      const double* __restrict__ ar = As + (k4 + lg) * kGLd + wi + li;
      const double* __restrict__ br = Bs + (k4 + lg) * kGLd + wj + li;
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = ar[16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = br[16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  double* __restrict__ pg = part + (long long)blockIdx.x * na * nb;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = i0 + wi + 16 * a + 4 * e + lg;
      if (i >= na) continue;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int j = j0 + wj + 16 * b + li;
        if (j < nb) pg[(long long)i * nb + j] = acc[a][b][e];
      }
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

// A (n x n, symmetric, lower triangle used) is factored as L L^T
// (right-looking, one workgroup); then Linv = L^{-1} (lower triangular, upper
// part zero), one column per thread by forward substitution.  status = 0, or
// k + 1 when the k-th pivot is not positive (A is not positive definite);
// Linv is not written then.  INLDS: the matrix is copied into LDS and
// factored there (n^2 doubles of dynamic LDS), else A is overwritten by L.
extern __shared__ __align__(16) double kx_chol_lds[];
template <bool INLDS>
__global__ void __launch_bounds__(1024) chol_inv(double* __restrict__ Ag, int n,
                                                 double* __restrict__ Linv, int* status) {
  const int t = threadIdx.x, nt = blockDim.x;
  double* A = Ag;
  if (INLDS) {
    A = kx_chol_lds;
    for (long long k = t; k < (long long)n * n; k += nt) A[k] = Ag[k];
  }
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
// 256 threads = 4 waves; wave w owns output rows 32 w .. 32 w + 31 of the
// 128-row block and all 64 points, as 2 x 4 blocks of 16 x 16 on
// v_mfma_f64_16x16x4f64 with A[m][k] = Cs[k][m] and B[k][n] = Xs[k][n].
template <class S>
__global__ void __launch_bounds__(256) combine(const double* __restrict__ C, long long ldv,
                                               long long ldk, int m, int n,
                                               const S* __restrict__ X, long long N, double alpha,
                                               S* __restrict__ Out) {
  typedef double v4d __attribute__((ext_vector_type(4)));
  __shared__ double Xs[kCK * kCR];
  __shared__ double Cs[kCK * (kCV + 2)];
  const int t = threadIdx.x;
  const int lane = t & 63, li = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const long long r0 = (long long)blockIdx.x * kCR;
  const int v0 = blockIdx.y * kCV;
  v4d acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0, 0, 0, 0};
  // staging: X rows k0 + t / 16, points 4 (t % 16) ..; C rows v0 + t / 2,
  // columns k0 + 8 (t % 2) ..
  const int xk = t >> 4, xr = (t & 15) * 4;
  const int cv = t >> 1, ck = (t & 1) * 8;
  // the next step's values are loaded into registers while this step is
  // multiplied
  double nx[4], nc[8];
  const bool vec = ((N * (long long)sizeof(S)) % 16 == 0) &&
                   (reinterpret_cast<unsigned long long>(X) & 15) == 0;
  auto fetch = [&](int k0) {
    const int k = k0 + xk;
    if (vec && k < n && r0 + xr + 4 <= N) {
      load4(X + (long long)k * N + r0 + xr, nx);
    } else {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const long long r = r0 + xr + b;
        nx[b] = (k < n && r < N) ? (double)X[(long long)k * N + r] : 0.0;
      }
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
#pragma unroll
    for (int k4 = 0; k4 < kCK; k4 += 4) {
      const double* __restrict__ cr = Cs + (k4 + lg) * (kCV + 2) + 32 * wave + li;
      const double* __restrict__ xr_ = Xs + (k4 + lg) * kCR + li;
      double av[2], bv[4];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = cr[16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = xr_[16 * b];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int v = v0 + 32 * wave + 16 * a + 4 * e + lg;
      if (v >= m) continue;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const long long r = r0 + 16 * b + li;
        if (r < N) Out[(long long)v * N + r] = (S)(alpha * acc[a][b][e]);
      }
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
  const size_t lds = (size_t)n * n * sizeof(double);
  int dev = 0, maxl = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&maxl, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
    (void)hipGetLastError();
    maxl = 0;
  }
  if (lds <= (size_t)maxl &&
      hipFuncSetAttribute((const void*)chol_inv<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds) == hipSuccess) {
    hipLaunchKernelGGL(chol_inv<true>, dim3(1), dim3(1024), lds, s, A, n, Linv, status);
  } else {
    (void)hipGetLastError();
    hipLaunchKernelGGL(chol_inv<false>, dim3(1), dim3(1024), 0, s, A, n, Linv, status);
  }
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

// ---- real form of complex fields (the compressed exchange of k-points)

namespace kx {
namespace {

__global__ void __launch_bounds__(256) realify_kernel(const double2* __restrict__ src, int n,
                                                     long long N, double2* __restrict__ dst) {
  const long long tot = (long long)n * N;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < tot;
       k += (long long)gridDim.x * blockDim.x) {
    const double2 z = src[k];
    dst[k] = z;
    dst[tot + k] = make_double2(-z.y, z.x);  // i z
  }
}

}  // namespace

hipError_t launch_realify(const double* src, int n, long long N, double* dst, hipStream_t s) {
  const long long tot = (long long)n * N;
  if (tot <= 0) return hipSuccess;
  const long long blocks = std::min<long long>((tot + 255) / 256, 8192);
  hipLaunchKernelGGL(realify_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     (const double2*)src, n, N, (double2*)dst);
  return hipGetLastError();
}

}  // namespace kx
