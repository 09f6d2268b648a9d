// Set-up kernels: the 1-D eigendecompositions of -L_k (Sec. III, Eq. (13))
// and the table f(lam1[a] + lam2[b] + lam3[c]) of Eqs. (17)-(19).
//
// Both run once per grid (or per kernel/omega) in FP64 on the device.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kx_internal.h"

namespace kx {
namespace {

constexpr int kJacobiThreads = 1024;

// Cyclic Jacobi with a round-robin ("tournament") ordering: in every round
// the m/2 index pairs are disjoint, so their rotations commute and are applied
// together, first to the rows of A, then to its columns and to V.  A sweep is
// m-1 rounds (m = n rounded up to even; a pair that touches the dummy index n
// is skipped).  A lives in global memory (row-major n x n, symmetric) and is
// driven to diagonal form; V accumulates the rotations.
//
// Rotation for (p, q) with a_pq != 0 (Golub & Van Loan, Sym.Schur2):
//   tau = (a_qq - a_pp) / (2 a_pq),  t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
//   c = 1/sqrt(1+t^2), s = t c;  A <- J^T A J,  V <- V J,
//   J = I except J_pp = J_qq = c, J_pq = s, J_qp = -s.
__global__ void __launch_bounds__(kJacobiThreads)
jacobi_kernel(double* __restrict__ A, double* __restrict__ V, int n, int max_sweeps, double rs,
              int keep_row, double* __restrict__ lam_pad, double* __restrict__ Vpad,
              double* __restrict__ VTpad, int np, double* __restrict__ diag_out) {
  __shared__ double cs[kMaxN / 2 + 1], sn[kMaxN / 2 + 1];
  __shared__ int pp[kMaxN / 2 + 1], qq[kMaxN / 2 + 1];
  __shared__ double lam_s[kMaxN];
  __shared__ int done;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int m = (n + 1) & ~1;
  const int half = m / 2;

  for (int idx = tid; idx < n * n; idx += nthr) V[idx] = (idx / n == idx % n) ? 1.0 : 0.0;
  __syncthreads();

  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) done = 1;  // cleared by any rotation of this sweep
    __syncthreads();
    for (int r = 0; r < m - 1; ++r) {
      if (tid < half) {
        // position 0 holds index 0; positions 1..m-1 rotate by one per round
        const int pa = tid, pb = m - 1 - tid;
        const int p0 = (pa == 0) ? 0 : 1 + (pa - 1 + r) % (m - 1);
        const int q0 = 1 + (pb - 1 + r) % (m - 1);
        int p = p0 < q0 ? p0 : q0, q = p0 < q0 ? q0 : p0;
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p * n + q];
          const double app = A[p * n + p], aqq = A[q * n + q];
          // rotate only while a_pq is significant relative to the diagonal
          if (fabs(apq) > 1e-300 && fabs(apq) > 1e-16 * sqrt(fabs(app * aqq))) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            done = 0;
          }
        } else {
          p = q = -1;
        }
        cs[tid] = c;
        sn[tid] = s;
        pp[tid] = p;
        qq[tid] = q;
      }
      __syncthreads();
      // rows: A[p,:] <- c A[p,:] - s A[q,:];  A[q,:] <- s A[p,:] + c A[q,:]
      for (int idx = tid; idx < half * n; idx += nthr) {
        const int k = idx / n, j = idx - k * n;
        const int p = pp[k], q = qq[k];
        if (p < 0 || sn[k] == 0.0) continue;
        const double c = cs[k], s = sn[k];
        const double ap = A[p * n + j], aq = A[q * n + j];
        A[p * n + j] = c * ap - s * aq;
        A[q * n + j] = s * ap + c * aq;
      }
      __syncthreads();
      // columns of A and V
      for (int idx = tid; idx < half * n; idx += nthr) {
        const int k = idx / n, i = idx - k * n;
        const int p = pp[k], q = qq[k];
        if (p < 0 || sn[k] == 0.0) continue;
        const double c = cs[k], s = sn[k];
        const double ap = A[i * n + p], aq = A[i * n + q];
        A[i * n + p] = c * ap - s * aq;
        A[i * n + q] = s * ap + c * aq;
        const double vp = V[i * n + p], vq = V[i * n + q];
        V[i * n + p] = c * vp - s * vq;
        V[i * n + q] = s * vp + c * vq;
      }
      __syncthreads();
      // the rotated entry is zero in exact arithmetic
      if (tid < half) {
        const int p = pp[tid], q = qq[tid];
        if (p >= 0 && sn[tid] != 0.0) {
          A[p * n + q] = 0.0;
          A[q * n + p] = 0.0;
        }
      }
      __syncthreads();
    }
    if (done) break;
  }

  // sort eigenvalues ascending (ties by index) and scatter into padded copies
  for (int i = tid; i < n; i += nthr) lam_s[i] = A[i * n + i];
  for (int idx = tid; idx < np * np; idx += nthr) {
    Vpad[idx] = 0.0;
    VTpad[idx] = 0.0;
  }
  for (int i = tid; i < np; i += nthr) lam_pad[i] = 0.0;
  __syncthreads();
  for (int t = tid; t < n; t += nthr) {
    const double lt = lam_s[t];
    int rank = 0;
    for (int u = 0; u < n; ++u) {
      const double lu = lam_s[u];
      rank += (lu < lt) || (lu == lt && u < t);
    }
    lam_pad[rank] = lt;
    for (int i = 0; i < n; ++i) {
      const double v = V[i * n + t] * (i == keep_row ? 1.0 : rs);
      Vpad[i * np + rank] = v;
      VTpad[rank * np + i] = v;
    }
  }
  if (tid == 0) diag_out[0] = (double)sweep;  // == max_sweeps: not converged
}

// f(lam1[a] + lam2[b] + lam3[c]) stored as F[c][a][b] (b fastest) with every
// mode index parity-blocked (even modes first, odd modes after pe), zero on
// padded indices.  Unscreened: 4 pi / lam.  Screened: (pi/w^2) g(x) with
// x = lam/(4 w^2), g(x) = -expm1(-x)/x, g(0) = 1 (equal to
// 4 pi (1 - exp(-lam/(4 w^2))) / lam without cancellation near lam = 0).
struct LamPtrs {
  const double* e[3];
  const double* o[3];
};

__device__ __forceinline__ bool blocked_lam(const LamPtrs& L, int axis, int idx, int me, int mo,
                                            int pe, double& lam) {
  if (idx < pe) {
    if (idx >= me) return false;
    lam = L.e[axis][idx];
    return true;
  }
  idx -= pe;
  if (idx >= mo) return false;
  lam = L.o[axis][idx];
  return true;
}

__global__ void ftable_kernel(LamPtrs L, Geom g, int kernel, double omega, ZeroMode zero,
                              double* __restrict__ F) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.fsize) return;
  const int b = (int)(idx % g.p2);
  const int a = (int)((idx / g.p2) % g.p1);
  const int c = (int)(idx / g.slab);
  double l1, l2, l3, f = 0.0;
  if (blocked_lam(L, 0, a, g.me1, g.mo1, g.pe1, l1) && blocked_lam(L, 1, b, g.me2, g.mo2, g.pe2, l2) &&
      blocked_lam(L, 2, c, g.me3, g.mo3, g.pe3, l3)) {
    const double lam = l1 + l2 + l3;
    if (kernel == KX_KERNEL_COULOMB) {
      f = (zero.on && lam <= zero.tol) ? zero.val : 4.0 * M_PI / lam;
    } else {
      const double x = lam / (4.0 * omega * omega);
      const double gx = (x == 0.0) ? 1.0 : -expm1(-x) / x;
      f = (M_PI / (omega * omega)) * gx;
    }
  }
  F[idx] = f;
}

}  // namespace

hipError_t launch_jacobi(double* A, double* V, int n, int max_sweeps, double rs, int keep_row,
                         double* lam_pad, double* Vpad, double* VTpad, int np, double* diag_out,
                         hipStream_t s) {
  hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(kJacobiThreads), 0, s, A, V, n, max_sweeps, rs,
                     keep_row, lam_pad, Vpad, VTpad, np, diag_out);
  return hipGetLastError();
}

hipError_t launch_ftable(const double* const lamE[3], const double* const lamO[3], const Geom& g,
                         int kernel, double omega, double* F, hipStream_t s, const ZeroMode& zero) {
  LamPtrs L;
  for (int k = 0; k < 3; ++k) {
    L.e[k] = lamE[k];
    L.o[k] = lamO[k];
  }
  const long long total = g.fsize;
  const int threads = 256;
  const long long blocks = (total + threads - 1) / threads;
  hipLaunchKernelGGL(ftable_kernel, dim3((unsigned)blocks), dim3(threads), 0, s, L, g, kernel,
                     omega, zero, F);
  return hipGetLastError();
}

}  // namespace kx
