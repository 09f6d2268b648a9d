// Brillouin-zone sampling (Sec. II): the pair problem of (m q, n k) carries
// Bloch boundary conditions at the wavevector k - q along the periodic axes.
//
// On a periodic axis of n nodes with the Bloch phase theta, the stencil
// operator factors as L(theta) = D M(theta) D^H, D = diag(e^{i theta x / n})
// (x the node index) and M(theta) the circulant whose entry p off the
// diagonal is w_p e^{i theta p / n} / h^2.  M(theta) commutes with the
// periodic Laplacian, so in its real eigenbasis (the folded even/odd blocks
// of the theta = 0 problem) -M(theta) is block diagonal: the even and the odd
// mode of one frequency couple through a 2 x 2 Hermitian block
//   [ A    i b ]
//   [ -i b  A  ]  = A I + b s,   s = [[0, i], [-i, 0]],
// and every other mode is a 1 x 1 block.  In three dimensions f(-L) then acts
// on groups of at most 2 x 2 x 2 spectral coefficients; with P(+-) = (I +- s)/2
// the projectors of s,
//   f = sum_{signs} f(sum_a A_a +- b_a) prod_a P_a(+-)
//     = sum_{S subset of the paired axes} c_S prod_{a in S} s_a,
//   c_S = 2^-d sum_{signs} f(...) prod_{a in S} sign_a,
// which the coupling kernel applies to the FP64 spectra of the real and the
// imaginary part of D^H rho.  The orbitals enter in the ramp-free form
// u_nk = e^{-2 pi i k.x / n} psi_nk, for which conj(u_mq) u_nk is exactly
// D^H conj(psi_mq) psi_nk at theta = 2 pi (k - q), and the update of Vx psi
// is accumulated in the same form.
#include <cmath>

#include "kx_internal.h"

namespace kx {
namespace {

__device__ __forceinline__ double f_of(int kernel, double omega, double lam) {
  if (kernel == KX_KERNEL_COULOMB) return 4.0 * M_PI / lam;
  const double x = lam / (4.0 * omega * omega);
  const double gx = (x == 0.0) ? 1.0 : -expm1(-x) / x;
  return (M_PI / (omega * omega)) * gx;
}

// full eigenvector `idx` (blocked index) of an axis at node i, from its upper half
__device__ __forceinline__ double vget(const BlochAxis& A, int idx, int i) {
  if (idx < A.pe) {
    const int j = i < A.me ? i : A.n - 1 - i;
    return A.VE[(size_t)j * A.pe + idx];
  }
  const int b = idx - A.pe;
  if (i < A.mo) return A.VO[(size_t)i * A.po + b];
  if (i >= A.n - A.mo) return -A.VO[(size_t)(A.n - 1 - i) * A.po + b];
  return 0.0;  // the middle node of odd n
}

__device__ __forceinline__ bool valid_idx(const BlochAxis& A, int idx) {
  return idx < A.pe ? idx < A.me : (idx - A.pe < A.mo && idx < A.pe + A.po);
}

// v1^T C v2 for the circulant C with C[i, (i + p) mod n] += c[p + m]
__device__ double circ_form(const BlochAxis& A, int i1, int i2, const double* c, int m) {
  double acc = 0.0;
  for (int i = 0; i < A.n; ++i) {
    const double a = vget(A, i1, i);
    if (a == 0.0) continue;
    double s = 0.0;
    for (int p = -m; p <= m; ++p) {
      int j = (i + p) % A.n;
      if (j < 0) j += A.n;
      s += c[p + m] * vget(A, i2, j);
    }
    acc += a * s;
  }
  return acc;
}

// Per class (theta = 2 pi (kq[ki] - kq[qi]), class = ki * K + qi) and axis,
// in the folded basis: A[idx], the diagonal of -M, and b[idx], the imaginary
// part of its entry (even, odd partner) at the even member; on a
// non-orthogonal cell also, for the first-derivative circulant with entries
// sgn(p) d_|p| e^{i theta p / n} / h, Q[idx] its (imaginary) diagonal and
// R[idx] the real part of its entry (even, odd partner) at the even member.
__global__ void bloch_table_kernel(BlochAxes B, const double* __restrict__ kq, int K, int pmax,
                                   double* __restrict__ tab) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y, cls = blockIdx.z;
  if (idx >= pmax) return;
  const BlochAxis& A = B.ax[a];
  double* tA = tab + ((size_t)cls * 3 + a) * kBlochTab * pmax;
  double av = 0.0, bv = 0.0, qv = 0.0, rv = 0.0;
  if (valid_idx(A, idx)) {
    if (!A.periodic) {
      av = idx < A.pe ? A.lamE[idx] : A.lamO[idx - A.pe];
    } else {
      const int ki = cls / K, qi = cls - ki * K;
      const double d = kq[ki * 3 + a] - kq[qi * 3 + a];  // theta / (2 pi)
      double cr[2 * kMaxStencil + 1], ci[2 * kMaxStencil + 1];
      const double ih2 = 1.0 / (A.h * A.h);
      for (int p = -B.m; p <= B.m; ++p) {
        double sn, cs;
        sincospi(2.0 * d * p / A.n, &sn, &cs);
        const double w = B.w[p < 0 ? -p : p];
        cr[p + B.m] = -w * cs * ih2;
        ci[p + B.m] = -w * sn * ih2;
      }
      av = circ_form(A, idx, idx, cr, B.m);
      const int o = A.part[idx];
      if (o >= 0 && idx < A.pe) bv = circ_form(A, idx, o, ci, B.m);
      if (B.nonorth) {
        const double ih = 1.0 / A.h;
        for (int p = -B.m; p <= B.m; ++p) {
          double sn, cs;
          sincospi(2.0 * d * p / A.n, &sn, &cs);
          const double dp = p == 0 ? 0.0 : (p > 0 ? B.d[p] : -B.d[-p]);
          cr[p + B.m] = dp * cs * ih;
          ci[p + B.m] = dp * sn * ih;
        }
        qv = circ_form(A, idx, idx, ci, B.m);
        if (o >= 0 && idx < A.pe) rv = circ_form(A, idx, o, cr, B.m);
      }
    }
  }
  tA[idx] = av;
  tA[pmax + idx] = bv;
  tA[2 * pmax + idx] = qv;
  tA[3 * pmax + idx] = rv;
}

// (P1, P2), P1 <= P2, of pair t in the row-major upper triangle of M states
__device__ __forceinline__ void pair_of(long long t, int M, int& P1, int& P2) {
  const double b = 2.0 * M + 1.0;
  long long r = (long long)((b - sqrt(b * b - 8.0 * (double)t)) * 0.5);
  if (r < 0) r = 0;
  if (r > M - 1) r = M - 1;
  auto start = [&](long long q) { return q * M - q * (q - 1) / 2; };
  while (r + 1 <= M - 1 && start(r + 1) <= t) ++r;
  while (r > 0 && start(r) > t) --r;
  P1 = (int)r;
  P2 = (int)(r + (t - start(r)));
}

__device__ __forceinline__ bool tile_valid(const PairMap& pm, int r, int c) {
  const int P1 = pm.r0 + r, P2 = pm.c0 + c;
  return P1 < pm.M && P2 < pm.M && P1 <= P2;
}

// (P1, P2) of item `item` of the tile
__device__ __forceinline__ void tile_pair(const PairMap& pm, int item, int& P1, int& P2) {
  int t = 0;
  P1 = P2 = 0;
  for (int r = 0; r < kTileR; ++r)
    for (int c = 0; c < kTileC; ++c)
      if (tile_valid(pm, r, c)) {
        if (t == item) {
          P1 = pm.r0 + r;
          P2 = pm.c0 + c;
          return;
        }
        ++t;
      }
}

__device__ __forceinline__ int class_of(const PairMap& pm, int item) {
  if (pm.M == 0) return pm.cls0;
  int P1, P2;
  tile_pair(pm, item, P1, P2);
  return (P2 / pm.norb) * pm.K + (P1 / pm.norb);  // k of the second state, q of the first
}

constexpr int kCoupleThreads = 256;
constexpr int kCoupleChunk = 8;  // items per thread of the coupling kernel

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
  return s;
}

// Y = f(-M) X on the coupled groups of the spectra of a chunk of items
// (real part in S[2 item], imaginary part in S[2 item + 1], fsize values
// each), in place.  One thread per group, the group named by its
// representative (per axis an unpaired mode or the even member of a pair);
// the coefficients c_S are recomputed only when the class changes along the
// chunk.  Re sum conj(X) Y per wave and item into part[item][wave].
template <bool NONORTH>
__global__ void __launch_bounds__(kCoupleThreads)
bloch_couple_kernel(BlochAxes B, Geom g, RepMap rm, const double* __restrict__ tab, int pmax,
                    int kernel, double omega, PairMap pm, int nitems, double* __restrict__ S,
                    double* __restrict__ part) {
  const long long gi = (long long)blockIdx.x * kCoupleThreads + threadIdx.x;
  const long long ngroups = (long long)rm.R[0] * rm.R[1] * rm.R[2];
  const bool live = gi < ngroups;
  const int nwaves = gridDim.x * (kCoupleThreads / 64);
  const int wave = (int)(gi >> 6);
  const int lane = threadIdx.x & 63;
  int idx[3] = {0, 0, 0}, prt[3] = {-1, -1, -1}, pmask = 0;
  int off[8];  // offsets inside one spectrum (< fsize)
  if (live) {
    const int r2 = (int)(gi % rm.R[1]);
    const int r1 = (int)((gi / rm.R[1]) % rm.R[0]);
    const int r3 = (int)(gi / ((long long)rm.R[0] * rm.R[1]));
    idx[0] = rm.rep[0][r1];
    idx[1] = rm.rep[1][r2];
    idx[2] = rm.rep[2][r3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      prt[a] = B.ax[a].part[idx[a]];
      if (prt[a] >= 0) pmask |= 1 << a;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int ja = (t & 1) ? prt[0] : idx[0], jb = (t & 2) ? prt[1] : idx[1];
      const int jc = (t & 4) ? prt[2] : idx[2];
      off[t] = (int)((long long)jc * g.slab + (long long)ja * g.p2 + jb);
    }
  }
  const int d = __builtin_popcount(pmask);
  const double scale = 1.0 / (double)(1 << d);
  const int i0 = blockIdx.y * kCoupleChunk;
  const int i1 = min(nitems, i0 + kCoupleChunk);
  int cur = -1;
  double c[8];
  for (int item = i0; item < i1; ++item) {
    const int cls = class_of(pm, item);
    double e = 0.0;
    if (live) {
      if (cls != cur) {
        cur = cls;
        const double* tb = tab + (size_t)cls * 3 * kBlochTab * pmax;
        double Aa[3], Ba[3], Qa[3], Ra[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const double* tA = tb + (size_t)a * kBlochTab * pmax;
          const bool pr = prt[a] >= 0;
          Aa[a] = pr ? 0.5 * (tA[idx[a]] + tA[prt[a]]) : tA[idx[a]];
          Ba[a] = pr ? tA[pmax + idx[a]] : 0.0;
          Qa[a] = Ra[a] = 0.0;
          if (NONORTH) {
            Qa[a] = pr ? 0.5 * (tA[2 * pmax + idx[a]] + tA[2 * pmax + prt[a]])
                       : tA[2 * pmax + idx[a]];
            Ra[a] = pr ? tA[3 * pmax + idx[a]] : 0.0;
          }
        }
        double f[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          // sign vector t: bit set = the -1 eigenvalue of s on that axis, where
          // -M acts as A + s b and the first-derivative block as i (Q - s R)
          double lam = 0.0;
          if (!NONORTH) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
              lam += Aa[a] + (((pmask >> a) & 1) ? (((t >> a) & 1) ? -Ba[a] : Ba[a]) : 0.0);
          } else {
            double q[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const double sg = ((t >> a) & 1) ? -1.0 : 1.0;
              lam += B.gm[a][a] * (Aa[a] + sg * Ba[a]);
              q[a] = Qa[a] - sg * Ra[a];
            }
            lam += 2.0 * (B.gm[0][1] * q[0] * q[1] + B.gm[0][2] * q[0] * q[2] +
                          B.gm[1][2] * q[1] * q[2]);
          }
          f[t] = (t & ~pmask) ? 0.0
                 : (kernel == KX_KERNEL_COULOMB && B.zero.on && lam <= B.zero.tol)
                     ? B.zero.val
                     : f_of(kernel, omega, lam);
        }
#pragma unroll
        for (int Sm = 0; Sm < 8; ++Sm) {
          double acc = 0.0;
#pragma unroll
          for (int t = 0; t < 8; ++t) acc += (__builtin_popcount(t & Sm) & 1) ? -f[t] : f[t];
          c[Sm] = (Sm & ~pmask) ? 0.0 : acc * scale;
        }
      }
      double* Sr = S + (size_t)(2 * item) * g.fsize;
      double* Si = Sr + g.fsize;
      double xr[8], xi[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        xr[t] = (t & ~pmask) ? 0.0 : Sr[off[t]];
        xi[t] = (t & ~pmask) ? 0.0 : Si[off[t]];
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        if (t & ~pmask) continue;
        double yr = 0.0, yi = 0.0;
#pragma unroll
        for (int Sm = 0; Sm < 8; ++Sm) {
          if (Sm & ~pmask) continue;
          // prod over a in Sm of (i if t_a = 0 else -i) = i^|Sm| (-1)^|t & Sm|
          double cr = c[Sm], ci = 0.0;
          const int q = __builtin_popcount(Sm) & 3;
          if (q == 1) { ci = cr; cr = 0.0; }
          else if (q == 2) { cr = -cr; }
          else if (q == 3) { ci = -cr; cr = 0.0; }
          if (__builtin_popcount(t & Sm) & 1) { cr = -cr; ci = -ci; }
          const int src = t ^ Sm;
          yr += cr * xr[src] - ci * xi[src];
          yi += cr * xi[src] + ci * xr[src];
        }
        e += xr[t] * yr + xi[t] * yi;
        Sr[off[t]] = yr;
        Si[off[t]] = yi;
      }
    }
    for (int o = 32; o > 0; o >>= 1) e += __shfl_down(e, o, 64);
    if (lane == 0) part[(size_t)item * nwaves + wave] = e;
  }
}

// e^{-2 pi i s} for s = sum_a t_a x_a / n_a, reduced to [-1/2, 1/2] first
__device__ __forceinline__ void ramp(const double* t, const Geom& g, long long x, double& c,
                                     double& sn) {
  const long long i1 = x % g.n1, i2 = (x / g.n1) % g.n2, i3 = x / ((long long)g.n1 * g.n2);
  double s = t[0] * (double)i1 / g.n1 + t[1] * (double)i2 / g.n2 + t[2] * (double)i3 / g.n3;
  s -= rint(s);
  double ss, cc;
  sincospi(2.0 * s, &ss, &cc);
  c = cc;
  sn = -ss;
}

// Z[2 b] + i Z[2 b + 1] = e^{-i theta.x / n} rho_b (rho interleaved complex)
__global__ void field_in_kernel(const double* __restrict__ rho, int nb, Geom g, BlochT th,
                                double* __restrict__ Z) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.N) return;
  double c, s;
  ramp(th.t, g, x, c, s);
  for (int b = 0; b < nb; ++b) {
    const double r = rho[2 * ((size_t)b * g.N + x)], i = rho[2 * ((size_t)b * g.N + x) + 1];
    Z[(size_t)(2 * b) * g.N + x] = c * r - s * i;
    Z[(size_t)(2 * b + 1) * g.N + x] = c * i + s * r;
  }
}

// phi_b = e^{+i theta.x / n} (Z[2 b] + i Z[2 b + 1]), interleaved complex
__global__ void field_out_kernel(const double* __restrict__ Z, int nb, Geom g, BlochT th,
                                 double* __restrict__ phi) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.N) return;
  double c, s;
  ramp(th.t, g, x, c, s);
  s = -s;
  for (int b = 0; b < nb; ++b) {
    const double r = Z[(size_t)(2 * b) * g.N + x], i = Z[(size_t)(2 * b + 1) * g.N + x];
    phi[2 * ((size_t)b * g.N + x)] = c * r - s * i;
    phi[2 * ((size_t)b * g.N + x) + 1] = c * i + s * r;
  }
}

// u_P = e^{-2 pi i k(P).x / n} psi_P into planar U (re, im fields per state);
// W = 0.  State P = k-point P / norb, band P % norb.
__global__ void orbitals_in_kernel(const double* __restrict__ psi, int M, int norb, Geom g,
                                   const double* __restrict__ kq, double* __restrict__ U,
                                   double* __restrict__ W) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.N) return;
  for (int P = 0; P < M; ++P) {
    double c, s;
    ramp(kq + 3 * (P / norb), g, x, c, s);
    const double r = psi[2 * ((size_t)P * g.N + x)], i = psi[2 * ((size_t)P * g.N + x) + 1];
    U[(size_t)(2 * P) * g.N + x] = c * r - s * i;
    U[(size_t)(2 * P + 1) * g.N + x] = c * i + s * r;
    W[(size_t)(2 * P) * g.N + x] = 0.0;
    W[(size_t)(2 * P + 1) * g.N + x] = 0.0;
  }
}

// (Vx psi)_P = e^{+2 pi i k(P).x / n} W_P, interleaved complex
__global__ void vx_out_kernel(const double* __restrict__ W, int M, int norb, Geom g,
                              const double* __restrict__ kq, double* __restrict__ vx) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.N) return;
  for (int P = 0; P < M; ++P) {
    double c, s;
    ramp(kq + 3 * (P / norb), g, x, c, s);
    s = -s;
    const double r = W[(size_t)(2 * P) * g.N + x], i = W[(size_t)(2 * P + 1) * g.N + x];
    vx[2 * ((size_t)P * g.N + x)] = c * r - s * i;
    vx[2 * ((size_t)P * g.N + x) + 1] = c * i + s * r;
  }
}

// The tile's states: its kTileC columns c0 + c in slots c, and its kTileR rows
// r0 + r in slots kTileC + r, or, on a tile of the diagonal (rows inside the
// columns), in the columns' slots.
__device__ __forceinline__ int row_slot(const PairMap& pm, int r) {
  return pm.r0 >= pm.c0 && pm.r0 < pm.c0 + kTileC ? pm.r0 - pm.c0 + r : kTileC + r;
}
constexpr int kSlots = kTileC + kTileR;

// Z[2 t] + i Z[2 t + 1] = conj(u_P1) u_P2 for the tile's pairs t; the tile's
// states are read once per grid point
__global__ void __launch_bounds__(256)
products_kernel(const double* __restrict__ U, PairMap pm, Geom g, double* __restrict__ Z) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.N) return;
  const size_t N = (size_t)g.N;
  double ur[kSlots], ui[kSlots];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    const int P = k < kTileC ? pm.c0 + k : pm.r0 + (k - kTileC);
    const bool ok = P < pm.M && (k < kTileC || row_slot(pm, k - kTileC) == k);
    ur[k] = ok ? U[2 * (size_t)P * N + x] : 0.0;
    ui[k] = ok ? U[(2 * (size_t)P + 1) * N + x] : 0.0;
  }
  int t = 0;
#pragma unroll
  for (int r = 0; r < kTileR; ++r) {
    const int rs = row_slot(pm, r);
#pragma unroll
    for (int c = 0; c < kTileC; ++c) {
      if (!tile_valid(pm, r, c)) continue;
      double ar = 0.0, ai = 0.0;
#pragma unroll
      for (int k = 0; k < kSlots; ++k)  // the row's slot (a register, not an indexed array)
        if (k == rs) {
          ar = ur[k];
          ai = ui[k];
        }
      Z[(size_t)(2 * t) * N + x] = ar * ur[c] + ai * ui[c];
      Z[(size_t)(2 * t + 1) * N + x] = ar * ui[c] - ai * ur[c];
      ++t;
    }
  }
}

// For the tile's pairs t in order, with phi' = Z[2 t] + i Z[2 t + 1]:
//   W_P2 -= occw_P1 u_P1 phi',  and for P1 != P2  W_P1 -= occw_P2 u_P2 conj(phi').
// Each thread owns one grid point of every state and holds the tile's
// states (u and the W accumulators) in registers, so every state receives
// its contributions in one fixed order (the tiles in launch order, the
// pairs of a tile in row-major order) whatever the batch size.
__global__ void __launch_bounds__(256)
update_kernel(const double* __restrict__ U, const double* __restrict__ Z, PairMap pm, Geom g,
              const double* __restrict__ occw, double* __restrict__ W) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.N) return;
  const size_t N = (size_t)g.N;
  double ur[kSlots], ui[kSlots], wr[kSlots], wi[kSlots], oc[kSlots];
  bool live[kSlots];
  int st[kSlots];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    const int P = k < kTileC ? pm.c0 + k : pm.r0 + (k - kTileC);
    live[k] = P < pm.M && (k < kTileC || row_slot(pm, k - kTileC) == k);
    st[k] = P;
    ur[k] = live[k] ? U[2 * (size_t)P * N + x] : 0.0;
    ui[k] = live[k] ? U[(2 * (size_t)P + 1) * N + x] : 0.0;
    wr[k] = live[k] ? W[2 * (size_t)P * N + x] : 0.0;
    wi[k] = live[k] ? W[(2 * (size_t)P + 1) * N + x] : 0.0;
    oc[k] = live[k] ? occw[P] : 0.0;
  }
  int t = 0;
#pragma unroll
  for (int r = 0; r < kTileR; ++r) {
    const int rs = row_slot(pm, r);
#pragma unroll
    for (int c = 0; c < kTileC; ++c) {
      if (!tile_valid(pm, r, c)) continue;
      const double pr = Z[(size_t)(2 * t) * N + x], pi = Z[(size_t)(2 * t + 1) * N + x];
      ++t;
      double ar = 0.0, ai = 0.0, o1 = 0.0;
#pragma unroll
      for (int k = 0; k < kSlots; ++k)
        if (k == rs) {
          ar = ur[k];
          ai = ui[k];
          o1 = oc[k];
        }
      // W_P2 -= occw_P1 u_P1 phi'
      wr[c] -= o1 * (ar * pr - ai * pi);
      wi[c] -= o1 * (ar * pi + ai * pr);
      if (pm.r0 + r == pm.c0 + c) continue;
      // W_P1 -= occw_P2 u_P2 conj(phi')
      const double dr = oc[c] * (ur[c] * pr + ui[c] * pi);
      const double di = oc[c] * (ui[c] * pr - ur[c] * pi);
#pragma unroll
      for (int k = 0; k < kSlots; ++k)
        if (k == rs) {
          wr[k] -= dr;
          wi[k] -= di;
        }
    }
  }
#pragma unroll
  for (int k = 0; k < kSlots; ++k)
    if (live[k]) {
      W[2 * (size_t)st[k] * N + x] = wr[k];
      W[(2 * (size_t)st[k] + 1) * N + x] = wi[k];
    }
}

// pairE[index(P1, P2)] = dV * sum of the coupling kernel's partials of item t (in order)
__global__ void __launch_bounds__(256) pair_sum_kernel(const double* __restrict__ part, int nblk,
                                                      PairMap pm, double dV,
                                                      double* __restrict__ pairE) {
  __shared__ double red[4];
  const int t = blockIdx.x;
  double s = 0.0;
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) s += part[(size_t)t * nblk + k];
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    int P1, P2;
    tile_pair(pm, t, P1, P2);
    pairE[(long long)P1 * pm.M - (long long)P1 * (P1 - 1) / 2 + (P2 - P1)] = dV * s;
  }
}

// E = -1/4 sum over ordered pairs of occw_P1 occw_P2 (rho, phi)_h: the
// unordered pairs P1 < P2 count twice
__global__ void __launch_bounds__(256) bloch_energy_kernel(const double* __restrict__ pairE, int M,
                                                          const double* __restrict__ occw,
                                                          double* __restrict__ ex) {
  __shared__ double red[4];
  const long long np = (long long)M * (M + 1) / 2;
  double s = 0.0;
  for (long long t = threadIdx.x; t < np; t += blockDim.x) {
    int P1, P2;
    pair_of(t, M, P1, P2);
    s += (P1 == P2 ? 1.0 : 2.0) * occw[P1] * occw[P2] * pairE[t];
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) *ex = -0.25 * s;
}

inline dim3 pts_grid(const Geom& g) { return dim3((unsigned)((g.N + 255) / 256)); }

}  // namespace

int bloch_couple_waves(const RepMap& rm) {
  const long long groups = (long long)rm.R[0] * rm.R[1] * rm.R[2];
  return (int)((groups + kCoupleThreads - 1) / kCoupleThreads) * (kCoupleThreads / 64);
}

hipError_t launch_bloch_table(const BlochAxes& B, const double* kq, int K, int pmax, double* tab,
                              hipStream_t s) {
  const dim3 grid((unsigned)((pmax + 63) / 64), 3, (unsigned)(K * K));
  hipLaunchKernelGGL(bloch_table_kernel, grid, dim3(64), 0, s, B, kq, K, pmax, tab);
  return hipGetLastError();
}

hipError_t launch_bloch_couple(const BlochAxes& B, const Geom& g, const RepMap& rm,
                               const double* tab, int pmax, int kernel, double omega,
                               const PairMap& pm, int nitems, double* S, double* part,
                               hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  const dim3 grid((unsigned)(bloch_couple_waves(rm) / (kCoupleThreads / 64)),
                  (unsigned)((nitems + kCoupleChunk - 1) / kCoupleChunk));
  if (B.nonorth)
    hipLaunchKernelGGL(bloch_couple_kernel<true>, grid, dim3(kCoupleThreads), 0, s, B, g, rm, tab,
                       pmax, kernel, omega, pm, nitems, S, part);
  else
    hipLaunchKernelGGL(bloch_couple_kernel<false>, grid, dim3(kCoupleThreads), 0, s, B, g, rm,
                       tab, pmax, kernel, omega, pm, nitems, S, part);
  return hipGetLastError();
}

hipError_t launch_bloch_fields(int dir, const Geom& g, const BlochT& th, int nb, const double* in,
                               double* out, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  if (dir == 0)
    hipLaunchKernelGGL(field_in_kernel, pts_grid(g), dim3(256), 0, s, in, nb, g, th, out);
  else
    hipLaunchKernelGGL(field_out_kernel, pts_grid(g), dim3(256), 0, s, in, nb, g, th, out);
  return hipGetLastError();
}

hipError_t launch_bloch_orbitals(int dir, const Geom& g, int M, int norb, const double* kq,
                                 const double* in, double* U, double* W, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  if (dir == 0)
    hipLaunchKernelGGL(orbitals_in_kernel, pts_grid(g), dim3(256), 0, s, in, M, norb, g, kq, U, W);
  else
    hipLaunchKernelGGL(vx_out_kernel, pts_grid(g), dim3(256), 0, s, (const double*)W, M, norb, g,
                       kq, U);
  return hipGetLastError();
}

hipError_t launch_bloch_products(const Geom& g, const double* U, const PairMap& pm, int nb,
                                 double* Z, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(products_kernel, pts_grid(g), dim3(256), 0, s, U, pm, g, Z);
  return hipGetLastError();
}

hipError_t launch_bloch_update(const Geom& g, const double* U, const double* Z, const PairMap& pm,
                               int nb, const double* occw, double* W, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(update_kernel, pts_grid(g), dim3(256), 0, s, U, Z, pm, g, occw, W);
  return hipGetLastError();
}

hipError_t launch_bloch_pair_sums(const double* part, int nblk, int nitems, const PairMap& pm,
                                  double dV, double* pairE, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(pair_sum_kernel, dim3(nitems), dim3(256), 0, s, part, nblk, pm, dV, pairE);
  return hipGetLastError();
}

hipError_t launch_bloch_energy(const double* pairE, int M, const double* occw, double* ex,
                               hipStream_t s) {
  hipLaunchKernelGGL(bloch_energy_kernel, dim3(1), dim3(256), 0, s, pairE, M, occw, ex);
  return hipGetLastError();
}

}  // namespace kx
