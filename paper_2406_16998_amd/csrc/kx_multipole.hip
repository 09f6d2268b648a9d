// Dirichlet boundary values from the multipole expansion of the Coulomb
// kernel for isolated systems (Sec. IV: the unscreened problem on a grid with
// vacuum on every side takes its boundary values from the expansion, enforced
// by modifying the right-hand side).
//
// With the stencil split into the nodes inside the grid (L_D) and those
// outside, -L phi = 4 pi rho at node x reads
//   -(L_D phi)(x) = 4 pi rho(x) + c(x),
//   c(x) = sum_k sum_{p: x + p e_k outside} (w_|p| / h_k^2) phi_ext(x + p e_k),
// so phi = f(-L_D)(rho + c / (4 pi)) with f = 4 pi / lam.  phi_ext is the
// expansion about a centre C of the field's charge,
//   phi_ext(r) = sum_{l <= lmax} sum_{m=0}^{l} (2 - [m = 0]) (l-m)!/(l+m)!
//                  (A_lm R^c_lm(d) + B_lm R^s_lm(d)) / |d|^(2l+1),   d = r - C,
//   A_lm + i B_lm = dV sum_r rho(r) (R^c_lm + i R^s_lm)(r - C),
// with the regular solid harmonics R^c_lm + i R^s_lm = Q_l^m(z, |d|^2) (x + i y)^m
// (r^l P_l^m(cos t) e^{i m p}), Q by the three-term recursion in l.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "kx_internal.h"

namespace kx {
namespace {

constexpr int kMomThreads = 256;
constexpr int kMomPoints = 16;  // points per thread per group

// moment index of (l, m, part): l^2 + 2 m - (m > 0) + part, part 0 = cos, 1 = sin
// (m = 0 has no sine part): (lmax + 1)^2 values in all
__host__ __device__ inline int mom_index(int l, int m, int part) {
  return l * l + (m == 0 ? 0 : 2 * m - 1 + part);
}

// R^c_lm, R^s_lm of d for l <= L and M0 <= m <= M1 into out[mom_index]
template <int L, int M0 = 0, int M1 = L>
__device__ __forceinline__ void solid_harmonics(double x, double y, double z, double* out) {
  const double r2 = x * x + y * y + z * z;
  double cm = 1.0, sm = 0.0;  // (x + i y)^m
  double dfac = 1.0;          // (2m - 1)!!
#pragma unroll
  for (int m = 0; m <= M1; ++m) {
    if (m > 0) {
      const double c2 = x * cm - y * sm, s2 = y * cm + x * sm;
      cm = c2;
      sm = s2;
      dfac *= (double)(2 * m - 1);
    }
    if (m < M0) continue;
    double q2 = 0.0, q1 = dfac;  // Q_{m-1}^m = 0, Q_m^m = (2m-1)!!
#pragma unroll
    for (int l = m; l <= L; ++l) {
      double q = q1;
      if (l > m) {
        // 1 / (l - m) folds to a constant of the unrolled recursion
        q = ((double)(2 * l - 1) * z * q1 - (double)(l + m - 1) * r2 * q2) * (1.0 / (double)(l - m));
        q2 = q1;
        q1 = q;
      }
      out[mom_index(l, m, 0)] = q * cm;
      if (m > 0) out[mom_index(l, m, 1)] = q * sm;
    }
  }
}

struct Coords {
  double h[3];  // spacings
  double c[3];  // expansion centre
};

// the moment indices of orders M0 <= m <= M1 (l <= L): [lo, lo + count)
// is not contiguous in mom_index, so kernels enumerate (l, m, part)
template <int L, int M0, int M1>
struct MRange {
  static constexpr int count() {
    int c = 0;
    for (int m = M0; m <= M1; ++m) c += (L - m + 1) * (m == 0 ? 1 : 2);
    return c;
  }
};

// partial moments of points [g * span, (g + 1) * span) of field b, for the
// orders M0 <= m <= M1 (a kernel per range keeps the harmonics and sums of
// one thread in few registers)
template <class S, int L, int M0, int M1>
__global__ void __launch_bounds__(kMomThreads)
moments_partial(const S* __restrict__ rho, Geom g, Coords cc, long long span,
                double* __restrict__ part) {
  constexpr int K = (L + 1) * (L + 1);
  constexpr int KR = MRange<L, M0, M1>::count();
  __shared__ double red[kMomThreads / 64][KR];
  const int grp = blockIdx.x, b = blockIdx.y, ngrp = gridDim.x;
  const S* __restrict__ f = rho + (long long)b * g.N;
  // the range's moment indices, in (m, l, part) order
  int kidx[KR];
  {
    int t = 0;
#pragma unroll
    for (int m = M0; m <= M1; ++m)
#pragma unroll
      for (int l = m; l <= L; ++l) {
        kidx[t++] = mom_index(l, m, 0);
        if (m > 0) kidx[t++] = mom_index(l, m, 1);
      }
  }
  double acc[KR];
#pragma unroll
  for (int k = 0; k < KR; ++k) acc[k] = 0.0;
  const long long p0 = (long long)grp * span, p1 = p0 + span < g.N ? p0 + span : g.N;
  // 32-bit node arithmetic (N <= 160^3): 64-bit division dominated the loop
  const unsigned n1 = (unsigned)g.n1, n12 = (unsigned)(g.n1 * g.n2);
  for (long long p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    const unsigned pu = (unsigned)p;
    const unsigned i3 = pu / n12, r12 = pu - i3 * n12;
    const unsigned i2 = r12 / n1, i1 = r12 - i2 * n1;
    const double v = (double)f[p];
    double R[K];
    solid_harmonics<L, M0, M1>(i1 * cc.h[0] - cc.c[0], i2 * cc.h[1] - cc.c[1],
                               i3 * cc.h[2] - cc.c[2], R);
#pragma unroll
    for (int k = 0; k < KR; ++k) acc[k] += v * R[kidx[k]];
  }
  // fixed-shape reduction: wave trees, then the waves in index order
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    double v = acc[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[wave][k] = v;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < KR; k += blockDim.x) {
    double s = 0.0;
    for (int w = 0; w < kMomThreads / 64; ++w) s += red[w][k];
    part[((long long)b * ngrp + grp) * K + kidx[k]] = s;
  }
}

// moments[b][k] = dV * sum over groups in order
// moments[b][k] = dV * sum over groups: four fixed segments of the groups,
// each summed in order, then the segments in order
constexpr int kRedSeg = 4;
__global__ void __launch_bounds__(64 * kRedSeg) moments_reduce(const double* __restrict__ part,
                                                               int ngrp, int K, double dV,
                                                               double* __restrict__ mom) {
  __shared__ double seg[kRedSeg][64];
  const int b = blockIdx.x, k = threadIdx.x & 63, sg = threadIdx.x >> 6;
  const int per = (ngrp + kRedSeg - 1) / kRedSeg;
  const int q0 = sg * per, q1 = min(ngrp, q0 + per);
  double s = 0.0;
  if (k < K)
    for (int q = q0; q < q1; ++q) s += part[((long long)b * ngrp + q) * K + k];
  seg[sg][k] = s;
  __syncthreads();
  if (sg == 0 && k < K) {
    double t = 0.0;
    for (int i = 0; i < kRedSeg; ++i) t += seg[i][k];
    mom[(long long)b * K + k] = dV * t;
  }
}

struct Stencil {
  double w[13];  // w_0 .. w_m of the second-derivative stencil
  int m;
  double wl[(kMaxMultipoleL + 1) * (kMaxMultipoleL + 2) / 2];  // (2 - [m=0]) (l-m)!/(l+m)!
};

template <int L>
__device__ __forceinline__ double expanded_potential(const double* __restrict__ mom,
                                                     const Stencil& st, double x, double y,
                                                     double z) {
  constexpr int K = (L + 1) * (L + 1);
  double R[K];
  solid_harmonics<L>(x, y, z, R);
  const double r2 = x * x + y * y + z * z;
  const double ir2 = 1.0 / r2, ir = sqrt(ir2);
  double phi = 0.0, scale = ir;  // 1 / |d|^(2l+1)
  int t = 0;
#pragma unroll
  for (int l = 0; l <= L; ++l) {
    double sl = 0.0;
#pragma unroll
    for (int m = 0; m <= l; ++m, ++t) {
      double term = mom[mom_index(l, m, 0)] * R[mom_index(l, m, 0)];
      if (m > 0) term += mom[mom_index(l, m, 1)] * R[mom_index(l, m, 1)];
      sl += st.wl[t] * term;
    }
    phi += sl * scale;
    scale *= ir2;
  }
  return phi;
}

// dst = rho for every node of the fields (c is added afterwards, one axis at a
// time)
template <class S>
__global__ void __launch_bounds__(256)
copy_fields(const S* __restrict__ rho, S* __restrict__ dst, long long n) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x)
    dst[k] = rho[k];
}

// dst += c_k / (4 pi) for axis k: one thread per grid line along axis k of
// field b.  It evaluates the expansion at the m nodes beyond each end of its
// line, once each, then adds to every node x of the line within reach
//   sum_{p: x - q outside, q = x + p} (w_q / h_k^2) phi_ext(-p)        (low end)
// + sum_{p: x + q outside, q = n_k - 1 - x + p} (w_q / h_k^2) phi_ext(n_k - 1 + p).
// One launch per axis, so that lines of different axes never update a node
// at the same time.
template <class S, int L>
__global__ void __launch_bounds__(256)
boundary_axis(S* __restrict__ dst, Geom g, Coords cc, Stencil st,
              const double* __restrict__ moments, int k) {
  constexpr int K = (L + 1) * (L + 1);
  const int b = blockIdx.y;
  const double* __restrict__ mom = moments + (long long)b * K;
  const int n[3] = {g.n1, g.n2, g.n3};
  const int ka = k == 0 ? 1 : 0, kb = k == 2 ? 1 : 2;  // the other two axes
  const long long lines = (long long)n[ka] * n[kb];
  const long long line = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= lines) return;
  int idx[3];
  idx[ka] = (int)(line % n[ka]);
  idx[kb] = (int)(line / n[ka]);
  idx[k] = 0;
  const long long stride = k == 0 ? 1 : (k == 1 ? (long long)g.n1 : (long long)g.n1 * g.n2);
  const long long base = idx[0] + (long long)g.n1 * (idx[1] + (long long)g.n2 * idx[2]);
  double xyz[3] = {idx[0] * cc.h[0] - cc.c[0], idx[1] * cc.h[1] - cc.c[1],
                   idx[2] * cc.h[2] - cc.c[2]};
  const int m = st.m, nk = n[k];
  double lo[13], hi[13];  // phi_ext at -p and at n_k - 1 + p, p = 1..m
#pragma unroll 1
  for (int p = 1; p <= m; ++p) {
    xyz[k] = -p * cc.h[k] - cc.c[k];
    lo[p] = expanded_potential<L>(mom, st, xyz[0], xyz[1], xyz[2]);
    xyz[k] = (nk - 1 + p) * cc.h[k] - cc.c[k];
    hi[p] = expanded_potential<L>(mom, st, xyz[0], xyz[1], xyz[2]);
  }
  const double scale = 1.0 / (cc.h[k] * cc.h[k] * 4.0 * M_PI);
  S* __restrict__ o = dst + (long long)b * g.N + base;
#pragma unroll 1
  for (int x = 0; x < nk; ++x) {
    const int dl = x, dh = nk - 1 - x;  // distances to the two ends
    if (dl >= m && dh >= m) {
      x = nk - m - 1;  // skip to the first node the high end reaches
      continue;
    }
    double c = 0.0;
    for (int p = 1; p + dl <= m; ++p) c += st.w[p + dl] * lo[p];
    for (int p = 1; p + dh <= m; ++p) c += st.w[p + dh] * hi[p];
    S* q = o + x * stride;
    *q = (S)((double)*q + c * scale);
  }
}

template <class S, int L>
hipError_t launch_typed(const S* rho, S* dst, int nb, const Geom& g, const Coords& cc,
                        const Stencil& st, double dV, double* part, int ngrp, double* mom,
                        hipStream_t s) {
  constexpr int K = (L + 1) * (L + 1);
  const long long span = (g.N + ngrp - 1) / ngrp;
  // the orders m in two ranges of about equal size from L = 3 on
  constexpr int MS = L >= 3 ? (L + 1) / 2 - (L == 6 ? 1 : 0) : L;
  hipLaunchKernelGGL((moments_partial<S, L, 0, MS>), dim3(ngrp, nb), dim3(kMomThreads), 0, s, rho,
                     g, cc, span, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if constexpr (MS < L) {
    hipLaunchKernelGGL((moments_partial<S, L, MS + 1, L>), dim3(ngrp, nb), dim3(kMomThreads), 0, s,
                       rho, g, cc, span, part);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(moments_reduce, dim3(nb), dim3(64 * kRedSeg), 0, s, part, ngrp, K, dV, mom);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long tot = (long long)nb * g.N;
  const long long blocks = std::min<long long>((tot + 255) / 256, 8192);
  if (rho != dst) {  // (in place: rho is already there)
    hipLaunchKernelGGL(copy_fields<S>, dim3((unsigned)blocks), dim3(256), 0, s, rho, dst, tot);
    e = hipGetLastError();
  }
  const int n[3] = {g.n1, g.n2, g.n3};
  for (int k = 0; k < 3 && e == hipSuccess; ++k) {
    const long long lines = (long long)n[k == 0 ? 1 : 0] * n[k == 2 ? 1 : 2];
    hipLaunchKernelGGL((boundary_axis<S, L>), dim3((unsigned)((lines + 255) / 256), nb), dim3(256),
                       0, s, dst, g, cc, st, mom, k);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace

int multipole_groups(long long N) {
  long long grp = (N + (long long)kMomThreads * kMomPoints - 1) / ((long long)kMomThreads * kMomPoints);
  if (grp > kMaxMultipoleGroups) grp = kMaxMultipoleGroups;
  return grp < 1 ? 1 : (int)grp;
}

hipError_t launch_multipole_rhs(int storage, const void* rho, void* dst, int nb, const Geom& g,
                                const double h[3], const double centre[3], const double* w, int m,
                                int lmax, double* part, double* mom, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  if (lmax < 0 || lmax > kMaxMultipoleL || m < 1 || m > 12) return hipErrorInvalidValue;
  Coords cc;
  Stencil st;
  for (int k = 0; k < 3; ++k) {
    cc.h[k] = h[k];
    cc.c[k] = centre[k];
  }
  for (int p = 0; p <= 12; ++p) st.w[p] = p <= m ? w[p] : 0.0;
  st.m = m;
  int t = 0;
  for (int l = 0; l <= kMaxMultipoleL; ++l)
    for (int mm = 0; mm <= l; ++mm, ++t) {
      // (l - mm)! / (l + mm)! as a product, then the factor 2 for mm > 0
      double ratio = 1.0;
      for (int q = l - mm + 1; q <= l + mm; ++q) ratio /= (double)q;
      st.wl[t] = (mm == 0 ? 1.0 : 2.0) * ratio;
    }
  const double dV = h[0] * h[1] * h[2];
  const int ngrp = multipole_groups(g.N);
#define KX_L(LL)                                                                               \
  case LL:                                                                                     \
    return storage == KX_F64                                                                   \
               ? launch_typed<double, LL>((const double*)rho, (double*)dst, nb, g, cc, st, dV, \
                                          part, ngrp, mom, s)                                  \
               : launch_typed<float, LL>((const float*)rho, (float*)dst, nb, g, cc, st, dV,    \
                                         part, ngrp, mom, s);
  switch (lmax) {
    KX_L(0) KX_L(1) KX_L(2) KX_L(3) KX_L(4) KX_L(5) KX_L(6)
    default:
      return hipErrorInvalidValue;
  }
#undef KX_L
}

}  // namespace kx

// ---- the isolated-system exchange: pair fields and its energy
namespace kx {
namespace {

// Z[b] = psi_i psi_j for the pairs items[b] (FP64 fields of N values)
template <class S>
__global__ void __launch_bounds__(256) pair_fields_kernel(const S* __restrict__ psi,
                                                         const Item* __restrict__ items, int nb,
                                                         long long N, double* __restrict__ Z) {
  const int b = blockIdx.y;
  const Item it = items[b];
  const S* __restrict__ pi = psi + (long long)it.i * N;
  const S* __restrict__ pj = psi + (long long)it.j * N;
  double* __restrict__ zb = Z + (long long)b * N;
  for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < N;
       x += (long long)gridDim.x * blockDim.x)
    zb[x] = (double)pi[x] * (double)pj[x];
}

constexpr int kDotBlocks = 512;

// part[j * kDotBlocks + blk] = sum over this block's points of psi_j vx_j
template <class S>
__global__ void __launch_bounds__(256) vx_dot_kernel(const S* __restrict__ psi,
                                                    const S* __restrict__ vx, long long N,
                                                    double* __restrict__ part) {
  __shared__ double red[4];
  const int j = blockIdx.y;
  const S* __restrict__ a = psi + (long long)j * N;
  const S* __restrict__ v = vx + (long long)j * N;
  double s = 0.0;
  for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < N;
       x += (long long)gridDim.x * blockDim.x)
    s += (double)a[x] * (double)v[x];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)j * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// ex = 1/4 dV sum_j occ_j sum_blk part[j][blk]  (= E_x of the applied operator)
__global__ void __launch_bounds__(256) vx_energy_kernel(const double* __restrict__ part, int nblk,
                                                       int norb, const double* __restrict__ occ,
                                                       double dV, double* __restrict__ ex) {
  __shared__ double red[256];
  double s = 0.0;
  for (long long t = threadIdx.x; t < (long long)norb * nblk; t += blockDim.x)
    s += occ[t / nblk] * part[t];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *ex = 0.25 * dV * red[0];
}

}  // namespace

hipError_t launch_pair_fields(int storage, const void* psi, const Item* items, int nb, long long N,
                              double* Z, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  const dim3 grid((unsigned)std::min<long long>((N + 255) / 256, 1024), (unsigned)nb);
  if (storage == KX_F64)
    hipLaunchKernelGGL(pair_fields_kernel<double>, grid, dim3(256), 0, s, (const double*)psi, items,
                       nb, N, Z);
  else
    hipLaunchKernelGGL(pair_fields_kernel<float>, grid, dim3(256), 0, s, (const float*)psi, items,
                       nb, N, Z);
  return hipGetLastError();
}

int vx_energy_parts() { return kDotBlocks; }

hipError_t launch_vx_energy(int storage, const void* psi, const void* vx, int norb, long long N,
                            const double* occ, double dV, double* part, double* ex,
                            hipStream_t s) {
  if (norb <= 0) return hipSuccess;
  const dim3 grid(kDotBlocks, (unsigned)norb);
  if (storage == KX_F64)
    hipLaunchKernelGGL(vx_dot_kernel<double>, grid, dim3(256), 0, s, (const double*)psi,
                       (const double*)vx, N, part);
  else
    hipLaunchKernelGGL(vx_dot_kernel<float>, grid, dim3(256), 0, s, (const float*)psi,
                       (const float*)vx, N, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(vx_energy_kernel, dim3(1), dim3(256), 0, s, part, kDotBlocks, norb, occ, dV, ex);
  return hipGetLastError();
}

}  // namespace kx
