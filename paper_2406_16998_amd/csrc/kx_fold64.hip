// FP64 transform kernels for X = f(L) B (Sec. III, Eqs. (20)-(21)) and the
// exchange operator built on it (Sec. II, Eqs. (3)-(5)), on folded
// (even/odd) eigenvector blocks: every mode product of Eq. (21) is done as two
// half-size products (see kx_internal.h), halving the flops.
//
// Three passes per batch of independent items (an item is one field for
// apply_fL, or one orbital pair (i, j) for the exchange):
//
//   forward  per (item, z-slab):  S = rho[z] or psi_i[z] psi_j[z], folded in
//            y and x into four quadrants S_pq (p: y parity, q: x parity);
//            T'_pq = S_pq^T V2p (mode 2),  T1[a_q][b_p] = V1q^T T'_pq (mode 1)
//   pencil   per (item, 16 blocked columns (a, b)): fold T1 in z,
//            B~ = V3e^T T1_e, V3o^T T1_o (mode 3), e += F B~^2, X~ = F B~
//            (Hadamard product of Eq. (21b)), T2 = unfold(V3e X~_e, V3o X~_o)
//   inverse  per (item, z-slab):  W_pq = T2_pq^T V1q^T (mode 1 back),
//            Q_pq = V2p W_pq (mode 2 back), phi = unfold in y and x; then
//            phi -> output, or (Vx psi)_j -= occ_i phi psi_i and, for i != j,
//            (Vx psi)_i -= occ_j phi psi_j (Eq. (3))
//
// All contractions run on v_mfma_f64_16x16x4f64.  Operand layout on gfx950
// (lane l = 0..63, li = l % 16, lg = l / 16; measured):
//   A (16 x 4):  lane l holds A[li][lg]
//   B (4 x 16):  lane l holds B[lg][li]
//   D (16 x 16): lane l, element r holds D[4*r + lg][li]
// So element r of an accumulator tile t is, lane for lane, the B operand of
// the k-step that covers k = 16 t + 4 r .. 16 t + 4 r + 3: the second product
// of each pass consumes the first one's accumulators directly, and the
// intermediate between them never leaves registers.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kx_internal.h"

namespace kx {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dbl4 mfma_f64(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr dbl4 kZero4 = {0.0, 0.0, 0.0, 0.0};
constexpr int kFwdPos = 2;  // staged fold positions per thread per chunk (forward)
constexpr int kInvEl = 8;   // staged elements per thread per chunk (inverse)

// Per-wave MFMA building blocks with compile-time tile counts, so that the
// unrolled accumulator updates carry no runtime guards.
template <int NTQ>
__device__ __forceinline__ void fwd_k_step(dbl4* acc1, const double* __restrict__ arow,
                                           double bop) {
#pragma unroll
  for (int t = 0; t < NTQ; ++t) acc1[t] = mfma_f64(arow[kTile * t], bop, acc1[t]);
}

template <int NTQ>
__device__ __forceinline__ void fwd_mode1(const dbl4* acc1, dbl4* acc2,
                                          const double* __restrict__ V1q, int ldq, int lg, int li) {
#pragma unroll
  for (int t = 0; t < NTQ; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double bop = acc1[t][r];
      const double* __restrict__ vrow = V1q + (kTile * t + 4 * r + lg) * ldq + li;
#pragma unroll
      for (int u = 0; u < NTQ; ++u) acc2[u] = mfma_f64(vrow[kTile * u], bop, acc2[u]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <int NTQ>
__device__ __forceinline__ void fwd_store(const dbl4* acc2, double* __restrict__ Tzb, int p2,
                                          int lg) {
#pragma unroll
  for (int u = 0; u < NTQ; ++u) {
#pragma unroll
    for (int r = 0; r < 4; ++r) Tzb[(unsigned)(kTile * u + 4 * r + lg) * p2] = acc2[u][r];
  }
}

// ================================================================ forward
// Workgroup: `slabs` z-slabs; per slab one wave per (x parity q, y parity p,
// 16-wide b strip).  With qsplit == 2 a workgroup covers one x parity only
// (blockIdx.z).  The folded quadrants of S are staged through LDS in chunks
// of kc folded rows, double-buffered through registers.
template <int NT, bool OFULL, int MODE, bool VLDS, int MT>
__global__ void __launch_bounds__(MT)
forward_fold(Geom g, Eig e, const double* __restrict__ src, const Item* __restrict__ items,
             double* __restrict__ T, int slabs, int kc, int qsplit) {
  extern __shared__ double lds[];
  const int tid = threadIdx.x;
  const int lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nb = g.p2 / kTile, nbe = g.pe2 / kTile;
  const int wps = (qsplit == 1 ? 2 : 1) * nb;  // waves per slab
  const int s = wave / wps;
  const int w = wave - s * wps;
  const int q = (qsplit == 1) ? (w / nb) : (int)blockIdx.z;
  const int rem = w % nb;
  const int p = rem < nbe ? 0 : 1;
  const int b0 = (p == 0 ? rem : rem - nbe) * kTile;
  const int z = blockIdx.x * slabs + s;
  const bool zin = z < g.n3;
  const int it = blockIdx.y;
  const Item item = items[it];

  // staged row layout: [p][kc][wrow], quadrant q at column qcol(q)
  const int q_lo = (qsplit == 1) ? 0 : (int)blockIdx.z;
  const int q_hi = (qsplit == 1) ? 2 : q_lo + 1;
  const int wrow = (qsplit == 1) ? g.p1 : (q_lo == 0 ? g.pe1 : g.po1);
  auto qcol = [&](int qq) { return (qsplit == 1 && qq == 1) ? g.pe1 : 0; };
  const int celems = 2 * kc * wrow;
  // LDS: [V1 blocks (VLDS)] [slabs][2 buffers][celems]
  double* __restrict__ vE = lds;
  double* __restrict__ vO = lds + ((qsplit == 1 || q_lo == 0) ? g.pe1 * g.pe1 : 0);
  const int vsize = (qsplit == 1) ? (g.pe1 * g.pe1 + g.po1 * g.po1)
                                  : (q_lo == 0 ? g.pe1 * g.pe1 : g.po1 * g.po1);
  double* __restrict__ sb = lds + (VLDS ? vsize : 0) + (size_t)s * 2 * celems;
  if (VLDS) {
    if (q_lo == 0)
      for (int idx = tid; idx < g.pe1 * g.pe1; idx += blockDim.x) vE[idx] = e.VE[0][idx];
    if (q_hi == 2)
      for (int idx = tid; idx < g.po1 * g.po1; idx += blockDim.x) vO[idx] = e.VO[0][idx];
  }

  // fold staging: positions (yy, x') of the even-even range, kFwdPos per thread
  const int sthreads = wps * 64;
  const int stid = tid - s * sthreads;
  const long long zoff = (long long)(zin ? z : 0) * g.n1 * g.n2;
  const double* __restrict__ s0 = src + (long long)item.i * g.N + zoff;
  const double* __restrict__ s1 = src + (long long)(MODE == 1 ? item.j : item.i) * g.N + zoff;
  const int npos = kc * g.pe1;
  double ra[kFwdPos][4], rb[kFwdPos][4];
  auto fetch = [&](int y0) {
#pragma unroll
    for (int k = 0; k < kFwdPos; ++k) {
      const int pos = stid + k * sthreads;
      const int yy = pos / g.pe1, xp = pos - yy * g.pe1;
      const int y = y0 + yy, ym = g.n2 - 1 - y, xm = g.n1 - 1 - xp;
      const bool in = zin && pos < npos && y < g.me2 && xp < g.me1;
      const bool hx = in && xp < g.mo1, hy = in && y < g.mo2;
      const int o[4] = {y * g.n1 + xp, y * g.n1 + xm, ym * g.n1 + xp, ym * g.n1 + xm};
      const bool ok[4] = {in, hx, hy, hx && hy};
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        ra[k][m] = ok[m] ? s0[o[m]] : 0.0;
        if (MODE == 1) rb[k][m] = ok[m] ? s1[o[m]] : 0.0;
      }
    }
  };
  auto stash = [&](double* buf, int ybase) {
#pragma unroll
    for (int k = 0; k < kFwdPos; ++k) {
      const int pos = stid + k * sthreads;
      if (pos >= npos) continue;
      const int yy = pos / g.pe1, xp = pos - yy * g.pe1;
      double v[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) v[m] = (MODE == 1) ? ra[k][m] * rb[k][m] : ra[k][m];
      // v = S at (y,x), (y,x*), (y*,x), (y*,x*); fold sums / differences
      const double sx0 = v[0] + v[1], dx0 = v[0] - v[1];
      const double sx1 = v[2] + v[3], dx1 = v[2] - v[3];
      const int y = (pos / g.pe1) + ybase;
      const bool xo = xp < g.mo1, yo = y < g.mo2;  // odd folds exist here
      for (int qq = q_lo; qq < q_hi; ++qq) {
        const int wq = qq == 0 ? g.pe1 : g.po1;
        if (xp >= wq) continue;
        const bool live = qq == 0 || xo;
        const double ve = !live ? 0.0 : (qq == 0 ? sx0 + sx1 : dx0 + dx1);         // y even
        const double vo = !(live && yo) ? 0.0 : (qq == 0 ? sx0 - sx1 : dx0 - dx1);  // y odd
        buf[(0 * kc + yy) * wrow + qcol(qq) + xp] = ve;
        buf[(1 * kc + yy) * wrow + qcol(qq) + xp] = vo;
      }
    }
  };

  constexpr int NTO = OFULL ? NT : NT - 1;  // odd-x tile count
  const bool qfull = q == 0 || OFULL;        // this wave's x parity has NT tiles
  const int mp2 = p == 0 ? g.me2 : g.mo2;            // folded y rows of parity p
  const double* __restrict__ V2p = p == 0 ? e.VE[1] : e.VO[1];
  const int ldp = p == 0 ? g.pe2 : g.po2;

  dbl4 acc1[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc1[t] = kZero4;
  const int nchunks = (g.me2 + kc - 1) / kc;
  fetch(0);
  stash(sb, 0);
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    const double* __restrict__ cur = sb + (c & 1) * celems;
    if (c + 1 < nchunks) fetch((c + 1) * kc);
    const int y0 = c * kc;
    for (int kk = 0; kk < kc; kk += 4) {
      const int y = y0 + kk + lg;
      const double bop = (y < mp2) ? V2p[y * ldp + b0 + li] : 0.0;
      const double* __restrict__ arow = cur + (p * kc + kk + lg) * wrow + qcol(q) + li;
      if (qfull)
        fwd_k_step<NT>(acc1, arow, bop);
      else
        fwd_k_step<NTO>(acc1, arow, bop);
    }
    if (c + 1 < nchunks) stash(sb + ((c + 1) & 1) * celems, (c + 1) * kc);
    __syncthreads();
  }

  // mode 1:  C[a][b] += A[a][x'] B[x'][b],  A = V1q^T, B = T' (registers)
  const double* __restrict__ V1q =
      VLDS ? (q == 0 ? (const double*)vE : (const double*)vO) : (q == 0 ? e.VE[0] : e.VO[0]);
  const int ldq = q == 0 ? g.pe1 : g.po1;
  dbl4 acc2[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) acc2[u] = kZero4;
  if (qfull)
    fwd_mode1<NT>(acc1, acc2, V1q, ldq, lg, li);
  else
    fwd_mode1<NTO>(acc1, acc2, V1q, ldq, lg, li);
  if (!zin) return;
  const int aoff = q == 0 ? 0 : g.pe1, boff = p == 0 ? 0 : g.pe2;
  double* __restrict__ Tzb =
      T + (long long)it * g.slot + (long long)z * g.slab + (long long)aoff * g.p2 + boff + b0 + li;
  if (qfull)
    fwd_store<NT>(acc2, Tzb, g.p2, lg);
  else
    fwd_store<NTO>(acc2, Tzb, g.p2, lg);
}

// ================================================================ pencil
// One wave per 16 blocked columns (a, b); the T1 column block is folded in z
// on load.  V3 blocks are resident in LDS (row stride +1 so that a column read
// across 16 lanes hits 16 banks) when they fit.
template <int NT, bool OFULL, bool VLDS, int MT>
__global__ void __launch_bounds__(MT)
pencil_fold(Geom g, Eig e, const double* __restrict__ F, double* __restrict__ T,
            double* __restrict__ epart) {
  constexpr int NTE = NT, NTO = OFULL ? NT : NT - 1;  // even / odd tile counts
  extern __shared__ double lds[];
  const int tid = threadIdx.x;
  const int lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nwaves = blockDim.x >> 6;
  const int nstrips = (int)(g.slab / kTile);
  const int qs = (int)blockIdx.x * nwaves + wave;
  const bool qin = qs < nstrips;
  const unsigned q0 = (unsigned)(qin ? qs : 0) * kTile;
  const unsigned slab = (unsigned)g.slab;
  const int it = blockIdx.y;
  double* __restrict__ Tb = T + (long long)it * g.slot + q0;  // wave-uniform base
  const int pe = g.pe3, po = g.po3;
  const int lde = pe + 1, ldo = po + 1;
  double* __restrict__ vE = lds;
  double* __restrict__ vO = lds + pe * lde;
  if (VLDS) {
    for (int idx = tid; idx < pe * pe; idx += blockDim.x) {
      const int zz = idx / pe, cc = idx - zz * pe;
      vE[zz * lde + cc] = e.VE[2][idx];
    }
    for (int idx = tid; idx < po * po; idx += blockDim.x) {
      const int zz = idx / po, cc = idx - zz * po;
      vO[zz * ldo + cc] = e.VO[2][idx];
    }
  }
  // folded column values for k-step k (z' = 4k + lg)
  double ce[4 * NT], co[4 * NT];
#pragma unroll
  for (int k = 0; k < 4 * NT; ++k) {
    const int zp = 4 * k + lg;
    const bool ie = qin && zp < g.me3, io = qin && zp < g.mo3;
    const double a = ie ? Tb[(unsigned)zp * slab + li] : 0.0;
    const double m = io ? Tb[(unsigned)(g.n3 - 1 - zp) * slab + li] : 0.0;
    ce[k] = a + m;
    co[k] = io ? a - m : 0.0;
  }
  if (VLDS) __syncthreads();

  dbl4 accE[NT], accO[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    accE[t] = kZero4;
    accO[t] = kZero4;
  }
  // mode 3 (folded):  C[c][q] += A[c][z'] B[z'][q],  A[c][z'] = V3p[z'][c]
#pragma unroll
  for (int k = 0; k < 4 * NT; ++k) {
    const int zp = 4 * k + lg;
    {
      const double* __restrict__ vr = VLDS ? (vE + zp * lde + li) : (e.VE[2] + zp * pe + li);
#pragma unroll
      for (int t = 0; t < NTE; ++t) accE[t] = mfma_f64(vr[kTile * t], ce[k], accE[t]);
    }
    if (4 * k < 16 * NTO) {
      const double* __restrict__ vr = VLDS ? (vO + zp * ldo + li) : (e.VO[2] + zp * po + li);
#pragma unroll
      for (int t = 0; t < NTO; ++t) accO[t] = mfma_f64(vr[kTile * t], co[k], accO[t]);
    }
    // keep operand reads within their k-step (bounds register pressure)
    __builtin_amdgcn_sched_barrier(0);
  }

  // Hadamard product with f(Lambda) and the pair-energy partial sum F B~^2
  const double* __restrict__ Fq = F + q0;
  double esum = 0.0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = kTile * t + 4 * r + lg;
      {
        const double f = qin ? Fq[(unsigned)c * slab + li] : 0.0;
        const double v = accE[t][r];
        esum += f * v * v;
        accE[t][r] = f * v;
      }
      if (t < NTO) {
        const double f = qin ? Fq[(unsigned)(pe + c) * slab + li] : 0.0;
        const double v = accO[t][r];
        esum += f * v * v;
        accO[t][r] = f * v;
      }
    }
  }

  // inverse mode 3 (folded):  C[z'][q] += A[z'][c] B[c][q],  A = V3p
  dbl4 outE[NT], outO[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    outE[u] = kZero4;
    outO[u] = kZero4;
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = kTile * t + 4 * r + lg;
      {
        const double bop = accE[t][r];
#pragma unroll
        for (int u = 0; u < NTE; ++u) {
          const double a = VLDS ? vE[(kTile * u + li) * lde + c] : e.VET[2][c * pe + kTile * u + li];
          outE[u] = mfma_f64(a, bop, outE[u]);
        }
      }
      if (t < NTO) {
        const double bop = accO[t][r];
#pragma unroll
        for (int u = 0; u < NTO; ++u) {
          const double a = VLDS ? vO[(kTile * u + li) * ldo + c] : e.VOT[2][c * po + kTile * u + li];
          outO[u] = mfma_f64(a, bop, outO[u]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // unfold: T2[z'] = P + Q, T2[n3-1-z'] = P - Q
  if (qin) {
#pragma unroll
    for (int u = 0; u < NTE; ++u) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int zp = kTile * u + 4 * r + lg;
        const double P = outE[u][r];
        const double Q = (u < NTO) ? outO[u][r] : 0.0;
        if (zp < g.me3) Tb[(unsigned)zp * slab + li] = P + Q;
        if (zp < g.mo3) Tb[(unsigned)(g.n3 - 1 - zp) * slab + li] = P - Q;
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) esum += __shfl_xor(esum, o);
  if (epart != nullptr && qin && lane == 0) epart[(long long)it * nstrips + qs] = esum;
}

// ================================================================ inverse
// acc1 layout: [q][p][t] flattened as acc1[(q * 2 + p) * NT + t]
template <int NT, int NTO>
__device__ __forceinline__ void inv_k_step(dbl4* acc1q, const double* __restrict__ arow, int pe2,
                                           double bop) {
#pragma unroll
  for (int t = 0; t < NT; ++t) acc1q[t] = mfma_f64(arow[kTile * t], bop, acc1q[t]);
#pragma unroll
  for (int t = 0; t < NTO; ++t)
    acc1q[NT + t] = mfma_f64(arow[pe2 + kTile * t], bop, acc1q[NT + t]);
}

// Q[p*2 + q] for output y' tile u:  Q_pq = sum_b V2p[y'][b] W_pq[b][x']
template <int NT, int NTO, bool HASO>
__device__ __forceinline__ void inv_mode2(const dbl4* acc1, dbl4* Q, int u,
                                          const double* __restrict__ VE2T,
                                          const double* __restrict__ VO2T, int pe2, int po2, int lg,
                                          int li) {
#pragma unroll
  for (int k = 0; k < 4; ++k) Q[k] = kZero4;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int b = kTile * t + 4 * r + lg;
      const double a = VE2T[b * pe2 + kTile * u + li];
      Q[0] = mfma_f64(a, acc1[(0 * 2 + 0) * NT + t][r], Q[0]);
      if (HASO) Q[1] = mfma_f64(a, acc1[(1 * 2 + 0) * NT + t][r], Q[1]);
      if (t < NTO && u < NTO) {
        const double ao = VO2T[b * po2 + kTile * u + li];
        Q[2] = mfma_f64(ao, acc1[(0 * 2 + 1) * NT + t][r], Q[2]);
        if (HASO) Q[3] = mfma_f64(ao, acc1[(1 * 2 + 1) * NT + t][r], Q[3]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// Workgroup: `slabs` z-slabs; per slab one wave per 16-wide x' strip, which
// computes all four (y parity p, x parity q) quadrants of its strip so that it
// can unfold phi in y and x.  Rows of T2 (both a parities) are staged through
// LDS in chunks of kc folded rows; the V2 blocks (transposed) sit in LDS.
template <int NT, bool OFULL, int MODE, bool VLDS, int MT>
__global__ void __launch_bounds__(MT)
inverse_fold(Geom g, Eig e, const double* __restrict__ T, const Item* __restrict__ items,
             const double* __restrict__ psi, const double* __restrict__ occ,
             double* __restrict__ dst, int slabs, int kc) {
  constexpr int NTO = OFULL ? NT : NT - 1;  // odd-y (b) tile count
  extern __shared__ double lds[];
  const int tid = threadIdx.x;
  const int lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nstr = g.pe1 / kTile;
  const int s = wave / nstr;
  const int x0 = (wave - s * nstr) * kTile;
  const int z = blockIdx.x * slabs + s;
  const bool zin = z < g.n3;
  const int it = blockIdx.y;
  const int pe2 = g.pe2, po2 = g.po2, p2 = g.p2;
  double* __restrict__ vET = lds;
  double* __restrict__ vOT = lds + pe2 * pe2;
  const int celems = 2 * kc * p2;  // [q][kc][p2]
  double* __restrict__ sb = lds + (VLDS ? pe2 * pe2 + po2 * po2 : 0) + (size_t)s * 2 * celems;
  if (VLDS) {
    for (int idx = tid; idx < pe2 * pe2; idx += blockDim.x) vET[idx] = e.VET[1][idx];
    for (int idx = tid; idx < po2 * po2; idx += blockDim.x) vOT[idx] = e.VOT[1][idx];
  }
  const int sthreads = nstr * 64;
  const int stid = tid - s * sthreads;
  const double* __restrict__ Tz = T + (long long)it * g.slot + (long long)(zin ? z : 0) * g.slab;
  double pa[kInvEl];
  auto fetch = [&](int a0) {
#pragma unroll
    for (int k = 0; k < kInvEl; ++k) {
      const int idx = stid + k * sthreads;
      const int row = idx / p2, col = idx - row * p2;  // row = qq*kc + aa
      const int qq = row / kc, aa = row - qq * kc;
      const int mq = qq == 0 ? g.me1 : g.mo1;
      const bool ok = zin && idx < celems && a0 + aa < mq;
      const unsigned a = (qq == 0 ? 0 : g.pe1) + a0 + aa;
      pa[k] = ok ? Tz[a * (unsigned)p2 + col] : 0.0;
    }
  };
  auto stash = [&](double* buf) {
#pragma unroll
    for (int k = 0; k < kInvEl; ++k) {
      const int idx = stid + k * sthreads;
      if (idx < celems) buf[idx] = pa[k];
    }
  };

  const int xp = x0 + li;
  const bool has_o = x0 < g.po1;  // this strip has odd-x columns (wave-uniform)
  dbl4 acc1[4 * NT];
#pragma unroll
  for (int k = 0; k < 4 * NT; ++k) acc1[k] = kZero4;

  const int nchunks = (g.me1 + kc - 1) / kc;
  fetch(0);
  stash(sb);
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    const double* __restrict__ cur = sb + (c & 1) * celems;
    if (c + 1 < nchunks) fetch((c + 1) * kc);
    const int a0 = c * kc;
    for (int kk = 0; kk < kc; kk += 4) {
      const int a = a0 + kk + lg;
      // B[k=a'][n=x'] = V1q[x'][a'] = V1qT[a'][x']
      const double be = (a < g.me1) ? e.VET[0][a * g.pe1 + xp] : 0.0;
      inv_k_step<NT, NTO>(acc1, cur + (kk + lg) * p2 + li, pe2, be);
      if (has_o) {
        const double bo = (a < g.mo1) ? e.VOT[0][a * g.po1 + xp] : 0.0;
        inv_k_step<NT, NTO>(acc1 + 2 * NT, cur + (kc + kk + lg) * p2 + li, pe2, bo);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if (c + 1 < nchunks) stash(sb + ((c + 1) & 1) * celems);
    __syncthreads();
  }

  // mode 2 back per y' tile u, then unfold in y and x and apply
  const bool xin = zin && xp < g.me1;
  const int xm = g.n1 - 1 - xp;
  const long long zoff = (long long)(zin ? z : 0) * g.n1 * g.n2;
  const Item item = items[it];
  const double* __restrict__ pi = psi + (long long)item.i * g.N + zoff;
  const double* __restrict__ pj = psi + (long long)(MODE == 1 ? item.j : item.i) * g.N + zoff;
  double* __restrict__ vj = dst + (long long)(MODE == 1 ? item.j : item.i) * g.N + zoff;
  double* __restrict__ vi = dst + (long long)item.i * g.N + zoff;
  const bool offdiag = MODE == 1 && item.i != item.j;
  const double oi = MODE == 1 ? occ[item.i] : 0.0;
  const double oj = MODE == 1 ? occ[item.j] : 0.0;
  const double* __restrict__ VE2T = VLDS ? (const double*)vET : e.VET[1];
  const double* __restrict__ VO2T = VLDS ? (const double*)vOT : e.VOT[1];
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    dbl4 Q[4];  // [p*2 + q]
    if (has_o)
      inv_mode2<NT, NTO, true>(acc1, Q, u, VE2T, VO2T, pe2, po2, lg, li);
    else
      inv_mode2<NT, NTO, false>(acc1, Q, u, VE2T, VO2T, pe2, po2, lg, li);
    if (!xin) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int yp = kTile * u + 4 * r + lg;
      if (yp >= g.me2) continue;
      const double ee = Q[0][r], eo = has_o ? Q[1][r] : 0.0;
      const double oe = u < NTO ? Q[2][r] : 0.0, oo = (has_o && u < NTO) ? Q[3][r] : 0.0;
      const int ym = g.n2 - 1 - yp;
      const bool hx = xp < g.mo1, hy = yp < g.mo2;
      const double ph[4] = {ee + eo + oe + oo, ee - eo + oe - oo, ee + eo - oe - oo,
                            ee - eo - oe + oo};
      const unsigned o[4] = {(unsigned)(yp * g.n1 + xp), (unsigned)(yp * g.n1 + xm),
                             (unsigned)(ym * g.n1 + xp), (unsigned)(ym * g.n1 + xm)};
      const bool ok[4] = {true, hx, hy, hx && hy};
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        if (!ok[m]) continue;
        if (MODE == 0) {
          vj[o[m]] = ph[m];
        } else {
          vj[o[m]] -= (oi * ph[m]) * pi[o[m]];
          if (offdiag) vi[o[m]] -= (oj * ph[m]) * pj[o[m]];
        }
      }
    }
  }
}

// ================================================================ energies
constexpr int kRedThreads = 256;

__device__ double block_sum_fixed(double v, double* red) {
  // fixed shape: wave tree, then waves summed in index order by thread 0
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  }
  return s;
}

__global__ void __launch_bounds__(kRedThreads)
pair_energy_kernel(const double* __restrict__ epart, int nstrips, const Item* __restrict__ items,
                   int norb, double dV, double* __restrict__ pair_e) {
  __shared__ double red[kRedThreads / 64];
  const int it = blockIdx.x;
  const double* __restrict__ p = epart + (long long)it * nstrips;
  double v = 0.0;
  for (int s = threadIdx.x; s < nstrips; s += blockDim.x) v += p[s];
  const double tot = block_sum_fixed(v, red);
  if (threadIdx.x == 0) {
    const Item item = items[it];
    const int i = item.i < item.j ? item.i : item.j;
    const int j = item.i < item.j ? item.j : item.i;
    pair_e[pair_index(i, j, norb)] = dV * tot;
  }
}

__global__ void __launch_bounds__(kRedThreads)
exchange_energy_kernel(const double* __restrict__ pair_e, const double* __restrict__ occ, int norb,
                       double* __restrict__ ex) {
  __shared__ double red[kRedThreads / 64];
  const long long npairs = (long long)norb * (norb + 1) / 2;
  double v = 0.0;
  int i = 0;
  long long row_end = norb;  // first pair index of row i+1
  for (long long p = threadIdx.x; p < npairs; p += blockDim.x) {
    while (p >= row_end) {
      ++i;
      row_end += norb - i;
    }
    const int j = (int)(p - (row_end - (norb - i))) + i;
    const double m = (i == j) ? 1.0 : 2.0;
    v += m * occ[i] * occ[j] * pair_e[p];
  }
  const double tot = block_sum_fixed(v, red);
  if (threadIdx.x == 0) ex[0] = -0.25 * tot;
}

// Dynamic LDS above 64 KiB has to be allowed per kernel.
template <class K>
void allow_lds(K kernel, size_t lds) {
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
}

// launch bounds (threads per workgroup) by register tiles NT, from each
// kernel's register footprint
constexpr int fwd_mt(int nt) { return nt <= 3 ? 1024 : (nt == 4 ? 768 : 640); }
constexpr int inv_mt(int nt) { return nt <= 2 ? 1024 : (nt == 3 ? 768 : 512); }
constexpr int pen_mt(int nt) { return nt <= 2 ? 1024 : 512; }

}  // namespace

// ================================================================ planning
Plan make_plan(const Geom& g, size_t max_lds) {
  Plan pl;
  const int ntx = g.pe1 / kTile;  // forward register tiles (x' / a)
  const int nty = g.pe2 / kTile;  // inverse register tiles (b / y')
  // forward: waves per slab = 2 * p2/16 (both x parities) or p2/16 (split)
  {
    SlabPlan& f = pl.fwd;
    const int maxw = fwd_mt(ntx) / 64;
    int wps = 2 * (g.p2 / kTile);
    f.qsplit = 1;
    if (wps > maxw) {
      f.qsplit = 2;
      wps /= 2;
    }
    f.slabs = 1;
    while (f.slabs * 2 * wps <= maxw && (f.slabs * wps) % 4 != 0) f.slabs *= 2;
    f.waves = f.slabs * wps;
    const int wrow = f.qsplit == 1 ? g.p1 : g.pe1;
    const size_t vb = (size_t)(f.qsplit == 1 ? g.pe1 * g.pe1 + g.po1 * g.po1 : g.pe1 * g.pe1) * 8;
    f.kc = 4;
    for (int c : {32, 16, 8, 4}) {
      if ((size_t)c * g.pe1 <= (size_t)kFwdPos * wps * 64 &&
          (size_t)f.slabs * 2 * 2 * c * wrow * 8 + vb <= max_lds) {
        f.kc = c;
        break;
      }
    }
    const size_t chunk = (size_t)f.slabs * 2 * 2 * f.kc * wrow * 8;
    f.vlds = chunk + vb <= max_lds;
    f.lds_bytes = chunk + (f.vlds ? vb : 0);
  }
  // inverse: waves per slab = pe1/16
  {
    SlabPlan& v = pl.inv;
    const int maxw = inv_mt(nty) / 64;
    const int wps = g.pe1 / kTile;
    v.slabs = 1;
    while ((v.slabs + 1) * wps <= maxw && (v.slabs * wps) % 4 != 0) ++v.slabs;
    v.waves = v.slabs * wps;
    const size_t vb = (size_t)(g.pe2 * g.pe2 + g.po2 * g.po2) * 8;
    v.kc = 4;
    for (int c : {16, 8, 4}) {
      if ((size_t)2 * c * g.p2 <= (size_t)kInvEl * wps * 64 &&
          (size_t)v.slabs * 2 * 2 * c * g.p2 * 8 + vb <= max_lds) {
        v.kc = c;
        break;
      }
    }
    const size_t chunk = (size_t)v.slabs * 2 * 2 * v.kc * g.p2 * 8;
    v.vlds = chunk + vb <= max_lds;
    v.lds_bytes = chunk + (v.vlds ? vb : 0);
  }
  {
    PencilPlan& p = pl.pen;
    p.waves = 8;
    const size_t vb = (size_t)(g.pe3 * (g.pe3 + 1) + g.po3 * (g.po3 + 1)) * 8;
    p.lds_bytes = vb <= max_lds ? vb : 0;
  }
  return pl;
}

#define KX_NT_CASES(MACRO) MACRO(1) MACRO(2) MACRO(3) MACRO(4) MACRO(5)

hipError_t launch_forward_f64(int mode, const Geom& g, const Plan& pl, const Eig& e,
                              const double* src, const Item* items, int nitems, double* T,
                              hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  const SlabPlan& p = pl.fwd;
  const dim3 grid((g.n3 + p.slabs - 1) / p.slabs, nitems, p.qsplit);
  const dim3 block(64 * p.waves);
  const size_t lb = p.lds_bytes;
  switch (g.pe1 / kTile) {
#define KX_CASE(NT)                                                                            \
  case NT: {                                                                                   \
    constexpr int MT = fwd_mt(NT);                                                             \
    auto k = forward_fold<NT, true, 1, true, MT>;                                              \
    const bool of = g.po1 == g.pe1;                                                            \
    if (mode == 1) {                                                                           \
      if (p.vlds) k = of ? forward_fold<NT, true, 1, true, MT> : forward_fold<NT, false, 1, true, MT>; \
      else k = of ? forward_fold<NT, true, 1, false, MT> : forward_fold<NT, false, 1, false, MT>; \
    } else {                                                                                   \
      if (p.vlds) k = of ? forward_fold<NT, true, 0, true, MT> : forward_fold<NT, false, 0, true, MT>; \
      else k = of ? forward_fold<NT, true, 0, false, MT> : forward_fold<NT, false, 0, false, MT>; \
    }                                                                                          \
    allow_lds(k, lb);                                                                          \
    hipLaunchKernelGGL(k, grid, block, lb, s, g, e, src, items, T, p.slabs, p.kc, p.qsplit);   \
    break;                                                                                     \
  }
    KX_NT_CASES(KX_CASE)
#undef KX_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pencil_f64(const Geom& g, const Plan& pl, const Eig& e, const double* F,
                             int nitems, double* T, double* epart, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  const long long nstrips = g.slab / kTile;
  const int w = pl.pen.waves;
  const dim3 grid((unsigned)((nstrips + w - 1) / w), nitems);
  const dim3 block(64 * w);
  const size_t lb = pl.pen.lds_bytes;
  switch (g.pe3 / kTile) {
#define KX_CASE(NT)                                                               \
  case NT: {                                                                      \
    constexpr int MT = pen_mt(NT);                                                \
    const bool of = g.po3 == g.pe3;                                               \
    auto k = lb > 0 ? (of ? pencil_fold<NT, true, true, MT> : pencil_fold<NT, false, true, MT>) \
                    : (of ? pencil_fold<NT, true, false, MT> : pencil_fold<NT, false, false, MT>); \
    allow_lds(k, lb);                                                             \
    hipLaunchKernelGGL(k, grid, block, lb, s, g, e, F, T, epart);                 \
    break;                                                                        \
  }
    KX_NT_CASES(KX_CASE)
#undef KX_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_inverse_f64(int mode, const Geom& g, const Plan& pl, const Eig& e,
                              const double* T, const Item* items, int nitems, const double* psi,
                              const double* occ, double* dst, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  const SlabPlan& p = pl.inv;
  const dim3 grid((g.n3 + p.slabs - 1) / p.slabs, nitems);
  const dim3 block(64 * p.waves);
  const size_t lb = p.lds_bytes;
  switch (g.pe2 / kTile) {
#define KX_CASE(NT)                                                                             \
  case NT: {                                                                                    \
    constexpr int MT = inv_mt(NT);                                                              \
    const bool of = g.po2 == g.pe2;                                                             \
    auto k = inverse_fold<NT, true, 1, true, MT>;                                               \
    if (mode == 1) {                                                                            \
      if (p.vlds) k = of ? inverse_fold<NT, true, 1, true, MT> : inverse_fold<NT, false, 1, true, MT>; \
      else k = of ? inverse_fold<NT, true, 1, false, MT> : inverse_fold<NT, false, 1, false, MT>; \
    } else {                                                                                    \
      if (p.vlds) k = of ? inverse_fold<NT, true, 0, true, MT> : inverse_fold<NT, false, 0, true, MT>; \
      else k = of ? inverse_fold<NT, true, 0, false, MT> : inverse_fold<NT, false, 0, false, MT>; \
    }                                                                                           \
    allow_lds(k, lb);                                                                           \
    hipLaunchKernelGGL(k, grid, block, lb, s, g, e, T, items, psi, occ, dst, p.slabs, p.kc);    \
    break;                                                                                      \
  }
    KX_NT_CASES(KX_CASE)
#undef KX_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pair_energy(const double* epart, int nstrips, const Item* items, int nitems,
                              int norb, double dV, double* pair_e, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(pair_energy_kernel, dim3(nitems), dim3(kRedThreads), 0, s, epart, nstrips,
                     items, norb, dV, pair_e);
  return hipGetLastError();
}

hipError_t launch_exchange_energy(const double* pair_e, const double* occ, int norb, double* ex,
                                  hipStream_t s) {
  hipLaunchKernelGGL(exchange_energy_kernel, dim3(1), dim3(kRedThreads), 0, s, pair_e, occ, norb,
                     ex);
  return hipGetLastError();
}

}  // namespace kx
