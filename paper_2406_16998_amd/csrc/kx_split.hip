// Split-BF16 transform kernels: the same three folded passes as kx_fold.inc,
// with every mode product computed from three-term bfloat16 splits of both
// operands on v_mfma_f32_16x16x16_bf16 (FP32 accumulation):
//
//   x ~ x0 + x1 + x2,  x0 = bf16(x), x1 = bf16(x - x0), x2 = bf16(x - x0 - x1)
//   A B ~ sum_{s + t <= 2} A_s B_t      (six products, smallest first)
//
// Products of two bf16 values are exact in FP32, so the error is the split
// truncation (~2^-24 relative) plus FP32 rounding of the accumulation.  The
// f(Lambda) scaling, the pair energies and the Vx psi update stay in FP64;
// intermediates between passes are FP32.
//
// Operand layout of the instruction (li = lane % 16, lg = lane / 16): lane l
// holds four k-consecutive values of A row li and of B column li in k-slots
// (lg, e), e = 0..3; the accumulator tile is D[4 lg + r][li] (measured).  Any
// assignment of k values to slots works as long as A and B use the same one;
// here slot (lg, e) of the k-step starting at k0 holds k = k0 + 4 lg + e, so
// accumulator tile t (rows 16 t + 4 lg + r) is, element for element, the B
// operand of the k-step starting at 16 t.
#include <hip/hip_runtime.h>

#include "kx_internal.h"

// The FP32 staging and update arithmetic below must round the same way in
// every launch shape (results are reproducible bit for bit across plans):
// no contraction of products and sums into fused operations.
#pragma clang fp contract(off)

#include "kx_epilogue.inc"

namespace kx {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

struct Split4 {
  s4 h[3];  // bf16 bit patterns of the three terms, 4 k-slots
};

__device__ __forceinline__ short bf16_bits(float x) {
  const __bf16 b = (__bf16)x;  // round to nearest even
  return __builtin_bit_cast(short, b);
}
__device__ __forceinline__ float bf16_value(short s) {
  return __builtin_bit_cast(float, (unsigned)(unsigned short)s << 16);
}

// The 16-bit type of the split terms.  BF16: 8-bit significands, FP32's
// exponent range, no scaling.  FP16: 11-bit significands and a 5-bit
// exponent, so the operands are brought into range by powers of two: the V
// blocks by 2^12 at set-up (|V| <= 1), every data operand by a power of two
// that puts its largest magnitude in [2^13, 2^14) (per item where the data
// are staged in chunks, per wave where the whole contraction range is in
// registers); the products are scaled back exactly.
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
struct BF16 {
  static constexpr bool kScaled = false;
  static constexpr float kVScale = 1.f;
  static __device__ __forceinline__ short bits(float x) { return bf16_bits(x); }
  static __device__ __forceinline__ float value(short b) { return bf16_value(b); }
  static __device__ __forceinline__ f4 mma(s4 a, s4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
};
struct F16 {
  static constexpr bool kScaled = true;
  static constexpr float kVScale = 4096.f;  // 2^12, the V blocks' scale
  static __device__ __forceinline__ short bits(float x) {
    return __builtin_bit_cast(short, (_Float16)x);  // round to nearest even
  }
  static __device__ __forceinline__ float value(short b) {
    return (float)__builtin_bit_cast(_Float16, b);
  }
  static __device__ __forceinline__ f4 mma(s4 a, s4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(h4, a),
                                                 __builtin_bit_cast(h4, b), c, 0, 0, 0);
  }
};

// x ~ x0 + x1 + x2, x0 = h(x), x1 = h(x - x0), x2 = h(x - x0 - x1); the
// residuals are exact in FP32.  sc: the operand's power-of-two scale (FP16).
template <class H>
__device__ __forceinline__ Split4 split4(float v0, float v1, float v2, float v3, float sc = 1.f) {
  Split4 o;
  const float v[4] = {v0, v1, v2, v3};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float r = H::kScaled ? v[e] * sc : v[e];
    const short a = H::bits(r);
    r -= H::value(a);
    const short b = H::bits(r);
    r -= H::value(b);
    const short c = H::bits(r);
    o.h[0][e] = a;
    o.h[1][e] = b;
    o.h[2][e] = c;
  }
  return o;
}

// 2^k with m 2^k in [2^13, 2^14); 1 when m is zero or not finite
__device__ __forceinline__ float pow2_scale(float m) {
  if (!(m > 0.f) || !(m <= 3.0e38f)) return 1.f;
  int ex;
  (void)frexpf(m, &ex);  // m = f 2^ex, f in [0.5, 1)
  return ldexpf(1.f, 14 - ex);
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ Split4 load_split(const short* __restrict__ p, int plane_stride) {
  // pre-split operand: 4 k-consecutive bf16 of each plane
  Split4 o;
#pragma unroll
  for (int s = 0; s < 3; ++s) o.h[s] = *reinterpret_cast<const s4*>(p + s * plane_stride);
  return o;
}

template <class H>
__device__ __forceinline__ f4 mma6(const Split4& a, const Split4& b, f4 c) {
  c = H::mma(a.h[2], b.h[0], c);
  c = H::mma(a.h[1], b.h[1], c);
  c = H::mma(a.h[0], b.h[2], c);
  c = H::mma(a.h[1], b.h[0], c);
  c = H::mma(a.h[0], b.h[1], c);
  c = H::mma(a.h[0], b.h[0], c);
  return c;
}
// largest magnitude over a wave's accumulator tiles
template <int N>
__device__ __forceinline__ float tiles_absmax(const f4* t) {
  float m = 0.f;
#pragma unroll
  for (int k = 0; k < N; ++k)
#pragma unroll
    for (int r = 0; r < 4; ++r) m = fmaxf(m, fabsf(t[k][r]));
  return wave_max(m);
}

constexpr f4 kZ = {0.f, 0.f, 0.f, 0.f};
constexpr int kSplitKc = 16; // staged K rows per chunk: one MFMA k-step

extern __shared__ __align__(16) float kx_split_lds[];

// ================================================================ forward
template <class H, int NTQ>
__device__ __forceinline__ void sf_k_step(f4* acc1, const float* __restrict__ arow, int wrow,
                                          const Split4& b, float sc) {
  // A slot (lg, e) = S[k0 + 4 lg + e][16 t + li]: arow points at row k0 + 4 lg
#pragma unroll
  for (int t = 0; t < NTQ; ++t) {
    const float* a = arow + kTile * t;
    acc1[t] = mma6<H>(split4<H>(a[0], a[wrow], a[2 * wrow], a[3 * wrow], sc), b, acc1[t]);
  }
}

template <class H, int NTQ>
__device__ __forceinline__ void sf_mode1(const f4* acc1, f4* acc2, const short* __restrict__ V1qT,
                                         int ldq, int pstride, int lg, int li, float sc) {
  // A[m = a][k = x'] = V1q[x'][a] = V1qT[a][x'];  B = split(acc1[t])
#pragma unroll
  for (int t = 0; t < NTQ; ++t) {
    const Split4 b = split4<H>(acc1[t][0], acc1[t][1], acc1[t][2], acc1[t][3], sc);
#pragma unroll
    for (int u = 0; u < NTQ; ++u) {
      const Split4 a = load_split(V1qT + (kTile * u + li) * ldq + kTile * t + 4 * lg, pstride);
      acc2[u] = mma6<H>(a, b, acc2[u]);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int NTQ>
__device__ __forceinline__ void sf_store(const f4* acc2, float* __restrict__ Tzb, int p2, int lg) {
#pragma unroll
  for (int u = 0; u < NTQ; ++u) {
#pragma unroll
    for (int r = 0; r < 4; ++r) Tzb[(unsigned)(kTile * u + 4 * lg + r) * p2] = acc2[u][r];
  }
}

// Workgroup layout as the FP32/FP64 forward pass (one wave per x parity q,
// y parity p, 16-wide b strip; `slabs` z-slabs); staged folded rows in
// chunks of kc (a multiple of 16).
// XST: some staged positions exceed the register budget (grids whose x
// extent is large against y) and are loaded directly in the stash step.
// omax (FP16): largest magnitude of each source vector (orbital or field).
template <class H, class S, int NT, bool OFULL, int MODE, bool XST, int MT>
__global__ void __launch_bounds__(MT, fwd_min_waves(NT))
split_forward(Geom g, EigS e, const S* __restrict__ src, const Item* __restrict__ items,
              float* __restrict__ T, int slabs, int kc, int qsplit, const float* __restrict__ omax) {
  float* lds = kx_split_lds;
  const int tid = threadIdx.x;
  const int lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nb = g.p2 / kTile, nbe = g.pe2 / kTile;
  const int wps = (qsplit == 1 ? 2 : 1) * nb;
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
  const int q_lo = (qsplit == 1) ? 0 : (int)blockIdx.z;
  const int q_hi = (qsplit == 1) ? 2 : q_lo + 1;
  const int wrow = (qsplit == 1) ? g.p1 : (q_lo == 0 ? g.pe1 : g.po1);
  auto qcol = [&](int qq) { return (qsplit == 1 && qq == 1) ? g.pe1 : 0; };
  const int celems = 2 * kc * wrow;
  float* __restrict__ sb = lds + (size_t)s * 2 * celems;

  const int sthreads = wps * 64;
  const int stid = tid - s * sthreads;
  const long long zoff = (long long)(zin ? z : 0) * g.n1 * g.n2;
  const S* __restrict__ s0 = src + (long long)item.i * g.N + zoff;
  const S* __restrict__ s1 = src + (long long)(MODE == 1 ? item.j : item.i) * g.N + zoff;
  const int npos = kc * g.pe1;
  // one staged position: the four mirror images (y, x), (y, n1-1-x),
  // (n2-1-y, x), (n2-1-y, n1-1-x) of the pair product
  // raw loads stay in storage precision until the stash step, so the
  // prefetch does not wait on them
  auto load_pos = [&](int pos, int yy, int xp, int y0, S* va, S* vb) {
    const int y = y0 + yy, ym = g.n2 - 1 - y, xm = g.n1 - 1 - xp;
    const bool in = zin && pos < npos && y < g.me2 && xp < g.me1;
    const bool hx = in && xp < g.mo1, hy = in && y < g.mo2;
    const int o[4] = {y * g.n1 + xp, y * g.n1 + xm, ym * g.n1 + xp, ym * g.n1 + xm};
    const bool ok[4] = {in, hx, hy, hx && hy};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      va[m] = ok[m] ? s0[o[m]] : S(0);
      if (MODE == 1) vb[m] = ok[m] ? s1[o[m]] : S(0);
    }
  };
  // FP32 arithmetic: the operands are split from FP32 values anyway
  auto store_pos = [&](float* buf, int yy, int xp, int ybase, const S* va, const S* vb) {
    float v[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] = (MODE == 1) ? (float)va[m] * (float)vb[m] : (float)va[m];
    const float sx0 = v[0] + v[1], dx0 = v[0] - v[1];
    const float sx1 = v[2] + v[3], dx1 = v[2] - v[3];
    const int y = yy + ybase;
    const bool xo = xp < g.mo1, yo = y < g.mo2;
    for (int qq = q_lo; qq < q_hi; ++qq) {
      const int wq = qq == 0 ? g.pe1 : g.po1;
      if (xp >= wq) continue;
      const bool live = qq == 0 || xo;
      const float ve = !live ? 0.f : (qq == 0 ? sx0 + sx1 : dx0 + dx1);
      const float vo = !(live && yo) ? 0.f : (qq == 0 ? sx0 - sx1 : dx0 - dx1);
      buf[(0 * kc + yy) * wrow + qcol(qq) + xp] = ve;
      buf[(1 * kc + yy) * wrow + qcol(qq) + xp] = vo;
    }
  };
  // this thread's staged positions are the same in every chunk
  int pyy[kFwdPos], pxp[kFwdPos];
#pragma unroll
  for (int k = 0; k < kFwdPos; ++k) {
    const int pos = stid + k * sthreads;
    pyy[k] = pos / g.pe1;
    pxp[k] = pos - pyy[k] * g.pe1;
  }
  S ra[kFwdPos][4], rb[kFwdPos][4];
  auto fetch = [&](int y0) {
#pragma unroll
    for (int k = 0; k < kFwdPos; ++k) load_pos(stid + k * sthreads, pyy[k], pxp[k], y0, ra[k], rb[k]);
  };
  auto stash = [&](float* buf, int y0) {
#pragma unroll
    for (int k = 0; k < kFwdPos; ++k) {
      const int pos = stid + k * sthreads;
      if (pos < npos) store_pos(buf, pyy[k], pxp[k], y0, ra[k], rb[k]);
    }
    if (XST) {
      for (int pos = stid + kFwdPos * sthreads; pos < npos; pos += sthreads) {
        S va[4], vb[4];
        const int yy = pos / g.pe1, xp = pos - yy * g.pe1;
        load_pos(pos, yy, xp, y0, va, vb);
        store_pos(buf, yy, xp, y0, va, vb);
      }
    }
  };

  constexpr int NTO = OFULL ? NT : NT - 1;
  const bool qfull = q == 0 || OFULL;
  // B[k = y'][n = b] = V2p[y'][b] = V2pT[b][y']: pre-split, k-contiguous rows
  const short* __restrict__ V2pT = p == 0 ? e.ET[1] : e.OT[1];
  const int ldp = p == 0 ? g.pe2 : g.po2;
  const int pst2 = ldp * ldp;

  // FP16: the folded products are bounded by four times the product of the
  // two vectors' largest magnitudes
  float sc1 = 1.f;
  if (H::kScaled)
    sc1 = pow2_scale(4.f * omax[item.i] * (MODE == 1 ? omax[item.j] : 1.f));
  f4 acc1[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc1[t] = kZ;
  const int nchunks = (g.me2 + kc - 1) / kc;
  fetch(0);
  stash(sb, 0);
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    const float* __restrict__ cur = sb + (c & 1) * celems;
    if (c + 1 < nchunks) fetch((c + 1) * kc);
    const int y0 = c * kc;
    for (int kk = 0; kk < kc && y0 + kk < ldp; kk += kTile) {
      // staged rows beyond the parity's length are zero; so are the padded V2 rows
      const Split4 b = load_split(V2pT + (b0 + li) * ldp + y0 + kk + 4 * lg, pst2);
      const float* __restrict__ arow = cur + (p * kc + kk + 4 * lg) * wrow + qcol(q) + li;
      if (qfull)
        sf_k_step<H, NT>(acc1, arow, wrow, b, sc1);
      else
        sf_k_step<H, NTO>(acc1, arow, wrow, b, sc1);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (c + 1 < nchunks) stash(sb + ((c + 1) & 1) * celems, (c + 1) * kc);
    __syncthreads();
  }

  const short* __restrict__ V1qT = q == 0 ? e.ET[0] : e.OT[0];
  const int ldq = q == 0 ? g.pe1 : g.po1;
  f4 acc2[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) acc2[u] = kZ;
  // FP16: acc1 carries 2^12 sc1; its B operand is rescaled per wave
  float m2 = 1.f, un2 = 1.f;
  if (H::kScaled) {
    const float un1 = 1.f / (H::kVScale * sc1);
    const float sc2 = pow2_scale(tiles_absmax<NT>(acc1) * un1);
    m2 = un1 * sc2;
    un2 = 1.f / (H::kVScale * sc2);
  }
  if (qfull)
    sf_mode1<H, NT>(acc1, acc2, V1qT, ldq, ldq * ldq, lg, li, m2);
  else
    sf_mode1<H, NTO>(acc1, acc2, V1qT, ldq, ldq * ldq, lg, li, m2);
  if (H::kScaled) {
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc2[u][r] *= un2;
  }
  if (!zin) return;
  const int aoff = q == 0 ? 0 : g.pe1, boff = p == 0 ? 0 : g.pe2;
  float* __restrict__ Tzb =
      T + (long long)it * g.slot + (long long)z * g.slab + (long long)aoff * g.p2 + boff + b0 + li;
  if (qfull)
    sf_store<NT>(acc2, Tzb, g.p2, lg);
  else
    sf_store<NTO>(acc2, Tzb, g.p2, lg);
}

// ================================================================ pencil
// tmax (FP16): per item, the largest magnitude of the result (float bits,
// raised with atomic maxima; zero before the launch).
// VL: the three planes of the pre-split V3 blocks (both orientations) are
// copied into LDS once per workgroup, rows padded by spen_pad elements so that
// the 16 rows an operand read touches start in different banks; otherwise
// every MFMA group reads them from global memory (L2).
template <class H, int NT, bool OFULL, bool VL, int MT>
__global__ void __launch_bounds__(MT)
split_pencil(Geom g, EigS e, const double* __restrict__ F, float* __restrict__ T,
             double* __restrict__ epart, unsigned* __restrict__ tmax) {
  constexpr int NTE = NT, NTO = OFULL ? NT : NT - 1;
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
  float* __restrict__ Tb = T + (long long)it * g.slot + q0;
  const int pe = g.pe3, po = g.po3;
  // operand sources: global (row stride pe / po, plane stride pe^2 / po^2) or LDS
  const short* sET = e.ET[2];
  const short* sOT = e.OT[2];
  const short* sE = e.E[2];
  const short* sO = e.O[2];
  int lde = pe, ldo = po, pse = pe * pe, pso = po * po;
  if constexpr (VL) {
    short* lds = reinterpret_cast<short*>(kx_split_lds);
    lde = pe + spen_pad();
    ldo = po + spen_pad();
    pse = pe * lde;
    pso = po * ldo;
    short* dET = lds;
    short* dOT = dET + 3 * pse;
    short* dE = dOT + 3 * pso;
    short* dO = dE + 3 * pse;
    // 4 bf16 (8 bytes) a thread per step; rows are multiples of 4 elements
    for (int idx = tid; idx < 3 * pe * pe / 4; idx += blockDim.x) {
      const int pl = idx / (pe * pe / 4), rem = idx - pl * (pe * pe / 4);
      const int row = rem / (pe / 4), col = (rem - row * (pe / 4)) * 4;
      *reinterpret_cast<s4*>(dET + pl * pse + row * lde + col) =
          *reinterpret_cast<const s4*>(e.ET[2] + pl * pe * pe + row * pe + col);
      *reinterpret_cast<s4*>(dE + pl * pse + row * lde + col) =
          *reinterpret_cast<const s4*>(e.E[2] + pl * pe * pe + row * pe + col);
    }
    for (int idx = tid; idx < 3 * po * po / 4; idx += blockDim.x) {
      const int pl = idx / (po * po / 4), rem = idx - pl * (po * po / 4);
      const int row = rem / (po / 4), col = (rem - row * (po / 4)) * 4;
      *reinterpret_cast<s4*>(dOT + pl * pso + row * ldo + col) =
          *reinterpret_cast<const s4*>(e.OT[2] + pl * po * po + row * po + col);
      *reinterpret_cast<s4*>(dO + pl * pso + row * ldo + col) =
          *reinterpret_cast<const s4*>(e.O[2] + pl * po * po + row * po + col);
    }
    sET = dET;
    sOT = dOT;
    sE = dE;
    sO = dO;
  }

  // folded column values, k-step t (z' = 16 t + 4 lg + e)
  Split4 be[NT], bo[NT];
  float sc3 = 1.f;
  if constexpr (H::kScaled) {  // FP16: one scale for the wave's folded columns
    float ce[NT][4], co[NT][4], m = 0.f;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int ee = 0; ee < 4; ++ee) {
        const int zp = kTile * t + 4 * lg + ee;
        const bool ie = qin && zp < g.me3, io = qin && zp < g.mo3;
        const float a = ie ? Tb[(unsigned)zp * slab + li] : 0.f;
        const float mm = io ? Tb[(unsigned)(g.n3 - 1 - zp) * slab + li] : 0.f;
        ce[t][ee] = a + mm;
        co[t][ee] = io ? a - mm : 0.f;
        m = fmaxf(m, fmaxf(fabsf(ce[t][ee]), fabsf(co[t][ee])));
      }
    sc3 = pow2_scale(wave_max(m));
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      be[t] = split4<H>(ce[t][0], ce[t][1], ce[t][2], ce[t][3], sc3);
      bo[t] = split4<H>(co[t][0], co[t][1], co[t][2], co[t][3], sc3);
    }
  } else {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      float ce[4], co[4];
#pragma unroll
      for (int ee = 0; ee < 4; ++ee) {
        const int zp = kTile * t + 4 * lg + ee;
        const bool ie = qin && zp < g.me3, io = qin && zp < g.mo3;
        const float a = ie ? Tb[(unsigned)zp * slab + li] : 0.f;
        const float m = io ? Tb[(unsigned)(g.n3 - 1 - zp) * slab + li] : 0.f;
        ce[ee] = a + m;
        co[ee] = io ? a - m : 0.f;
      }
      be[t] = split4<H>(ce[0], ce[1], ce[2], ce[3]);
      bo[t] = split4<H>(co[0], co[1], co[2], co[3]);
    }
  }
  const float un3 = 1.f / (H::kVScale * sc3);
  if constexpr (VL) __syncthreads();

  // mode 3 (folded):  C[c][q] += A[c][z'] B[z'][q],  A[c][z'] = V3p[z'][c] = V3pT[c][z']
  f4 accE[NT], accO[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    accE[t] = kZ;
    accO[t] = kZ;
  }
#pragma unroll
  for (int k = 0; k < NTE; ++k) {
#pragma unroll
    for (int t = 0; t < NTE; ++t) {
      const Split4 a = load_split(sET + (kTile * t + li) * lde + kTile * k + 4 * lg, pse);
      accE[t] = mma6<H>(a, be[k], accE[t]);
    }
    if (k < NTO) {
#pragma unroll
      for (int t = 0; t < NTO; ++t) {
        const Split4 a = load_split(sOT + (kTile * t + li) * ldo + kTile * k + 4 * lg, pso);
        accO[t] = mma6<H>(a, bo[k], accO[t]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }

  // Hadamard product with f(Lambda) (FP64) and the pair-energy partial sum
  const double* __restrict__ Fq = F + q0;
  double esum = 0.0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = kTile * t + 4 * lg + r;
      {
        const double f = qin ? Fq[(unsigned)c * slab + li] : 0.0;
        const double v = H::kScaled ? (double)(accE[t][r] * un3) : (double)accE[t][r];
        esum += f * v * v;
        accE[t][r] = (float)(f * v);
      }
      if (t < NTO) {
        const double f = qin ? Fq[(unsigned)(pe + c) * slab + li] : 0.0;
        const double v = H::kScaled ? (double)(accO[t][r] * un3) : (double)accO[t][r];
        esum += f * v * v;
        accO[t][r] = (float)(f * v);
      }
    }
  }
  // FP16: one scale for the wave's scaled coefficients
  float sc4 = 1.f;
  if (H::kScaled) sc4 = pow2_scale(fmaxf(tiles_absmax<NT>(accE), tiles_absmax<NT>(accO)));
  const float un4 = 1.f / (H::kVScale * sc4);

  // inverse mode 3 (folded):  C[z'][q] += A[z'][c] B[c][q],  A = V3p (rows z', k = c)
  f4 outE[NT], outO[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    outE[u] = kZ;
    outO[u] = kZ;
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    {
      const Split4 b = split4<H>(accE[t][0], accE[t][1], accE[t][2], accE[t][3], sc4);
#pragma unroll
      for (int u = 0; u < NTE; ++u) {
        const Split4 a = load_split(sE + (kTile * u + li) * lde + kTile * t + 4 * lg, pse);
        outE[u] = mma6<H>(a, b, outE[u]);
      }
    }
    if (t < NTO) {
      const Split4 b = split4<H>(accO[t][0], accO[t][1], accO[t][2], accO[t][3], sc4);
#pragma unroll
      for (int u = 0; u < NTO; ++u) {
        const Split4 a = load_split(sO + (kTile * u + li) * ldo + kTile * t + 4 * lg, pso);
        outO[u] = mma6<H>(a, b, outO[u]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  float tm = 0.f;
  if (qin) {
#pragma unroll
    for (int u = 0; u < NTE; ++u) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int zp = kTile * u + 4 * lg + r;
        const float P = H::kScaled ? outE[u][r] * un4 : outE[u][r];
        const float Q = (u < NTO) ? (H::kScaled ? outO[u][r] * un4 : outO[u][r]) : 0.f;
        if (zp < g.me3) Tb[(unsigned)zp * slab + li] = P + Q;
        if (zp < g.mo3) Tb[(unsigned)(g.n3 - 1 - zp) * slab + li] = P - Q;
        if (H::kScaled) tm = fmaxf(tm, fmaxf(fabsf(P + Q), fabsf(P - Q)));
      }
    }
  }
  if (H::kScaled) {  // vector atomic maximum of non-negative float bits
    tm = wave_max(tm);
    if (lane == 0 && tm > 0.f) atomicMax(tmax + it, __builtin_bit_cast(unsigned, tm));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) esum += __shfl_xor(esum, o);
  if (epart != nullptr && qin && lane == 0) epart[(long long)it * nstrips + qs] = esum;
}

// ================================================================ inverse
// acc1 layout [q][p][t] flattened as acc1[(q * 2 + p) * NT + t]
template <class H, int NT, int NTO>
__device__ __forceinline__ void si_k_step(f4* acc1q, const float* __restrict__ arow, int p2,
                                          int pe2, const Split4& b, float sc) {
  // A[m = b][k = a'] = T2[a'][b]: arow points at staged row k0 + 4 lg, column li
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const float* a = arow + kTile * t;
    acc1q[t] = mma6<H>(split4<H>(a[0], a[p2], a[2 * p2], a[3 * p2], sc), b, acc1q[t]);
  }
#pragma unroll
  for (int t = 0; t < NTO; ++t) {
    const float* a = arow + pe2 + kTile * t;
    acc1q[NT + t] = mma6<H>(split4<H>(a[0], a[p2], a[2 * p2], a[3 * p2], sc), b, acc1q[NT + t]);
  }
}

// lde / ldo: row strides of the even / odd V2 blocks (in global memory or
// LDS), pse / pso: their plane strides.
template <class H, int NT, int NTO, bool HASO>
__device__ __forceinline__ void si_mode2(const Split4* bs, f4* Q, int u, const short* __restrict__ VE2,
                                         const short* __restrict__ VO2, int lde, int ldo, int pse,
                                         int pso, int lg, int li) {
  // bs[(q * 2 + p) * NT + t] = split(acc1 tile); A[m = y'][k = b] = V2p[y'][b]
#pragma unroll
  for (int k = 0; k < 4; ++k) Q[k] = kZ;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const Split4 a = load_split(VE2 + (kTile * u + li) * lde + kTile * t + 4 * lg, pse);
    Q[0] = mma6<H>(a, bs[(0 * 2 + 0) * NT + t], Q[0]);
    if (HASO) Q[1] = mma6<H>(a, bs[(1 * 2 + 0) * NT + t], Q[1]);
    if (t < NTO && u < NTO) {
      const Split4 ao = load_split(VO2 + (kTile * u + li) * ldo + kTile * t + 4 * lg, pso);
      Q[2] = mma6<H>(ao, bs[(0 * 2 + 1) * NT + t], Q[2]);
      if (HASO) Q[3] = mma6<H>(ao, bs[(1 * 2 + 1) * NT + t], Q[3]);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// tmax (FP16): per item, the largest magnitude of T (float bits).
template <class H, class S, int NT, bool OFULL, int MODE, bool VL, int MT>
__global__ void __launch_bounds__(MT)
split_inverse(Geom g, EigS e, const float* __restrict__ T, const Item* __restrict__ items,
              const S* __restrict__ psi, const double* __restrict__ occ, S* __restrict__ dst,
              int slabs, int kc, const unsigned* __restrict__ tmax) {
  constexpr int NTO = OFULL ? NT : NT - 1;
  // LDS: [pre-split V2 blocks, rows padded (VL)] [slabs][staged chunks / phi plane]
  short* __restrict__ vE = reinterpret_cast<short*>(kx_split_lds);
  short* __restrict__ vO = vE + 3 * g.pe2 * sinv_ld(g.pe2);
  float* lds = kx_split_lds + (VL ? sinv_vbytes(g) / sizeof(float) : 0);
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
  const int celems = 2 * kc * p2;
  // this slab's LDS: the staged chunks, then the phi plane
  float* __restrict__ sb = lds + (size_t)s * inv_slab_elems(g, kTile, false);
  const float* __restrict__ Tz = T + (long long)it * g.slot + (long long)(zin ? z : 0) * g.slab;
  if (VL) {  // 8-byte pieces of the three planes of each block (visible after the first barrier)
    const int lde = sinv_ld(pe2), ldo = sinv_ld(po2);
    const int ne = 3 * pe2 * (pe2 / 4), no = 3 * po2 * (po2 / 4);
    for (int idx = tid; idx < ne + no; idx += blockDim.x) {
      const bool od = idx >= ne;
      const int k = od ? idx - ne : idx, w = od ? po2 : pe2, ld = od ? ldo : lde;
      const int row = k / (w / 4), c = k - row * (w / 4);  // row over planes x rows
      const s4 v = *reinterpret_cast<const s4*>((od ? e.O[1] : e.E[1]) + row * w + 4 * c);
      *reinterpret_cast<s4*>((od ? vO : vE) + row * ld + 4 * c) = v;
    }
  }
  // Staged chunk [q][kc][p2]: rows a0 .. a0 + kc of the even (q = 0) and odd
  // (q = 1) x-parity blocks of this slab, contiguous in T.  Copied global ->
  // LDS without registers, 1 KB per wave instruction (16 bytes a lane); the
  // padded rows of T hold zeros, and odd rows past po1 are never multiplied.
  const int segs = p2 / kTile;  // 1 KB segments per block of kc = 16 rows
  const int wv = wave - s * nstr;
  auto issue = [&](float* buf, int a0) {
    for (int sg = wv; sg < 2 * segs; sg += nstr) {
      const int qq = sg >= segs ? 1 : 0, k = sg - qq * segs;
      if (qq == 1 && a0 >= g.po1) break;
      const float* src = Tz + (size_t)((qq ? g.pe1 : 0) + a0) * p2 + k * 256 + lane * 4;
      __builtin_amdgcn_global_load_lds(src, buf + qq * kc * p2 + k * 256, 16, 0, 0);
    }
  };
  const int xp = x0 + li;
  const bool has_o = x0 < g.po1;
  f4 acc1[4 * NT];
#pragma unroll
  for (int k = 0; k < 4 * NT; ++k) acc1[k] = kZ;
  const int nchunks = (g.me1 + kc - 1) / kc;
  // B[k = a'][n = x'] = V1q[x'][a'] (rows x', k = a' contiguous; padded rows
  // are zero), loaded one chunk ahead so that the only wait on global memory
  // in the loop is the end-of-chunk wait for the staging copies
  Split4 be_n, bo_n = {};
  auto load_b = [&](int a0) {
    be_n = load_split(e.E[0] + xp * g.pe1 + a0 + 4 * lg, g.pe1 * g.pe1);
    if (has_o && a0 < g.po1) bo_n = load_split(e.O[0] + xp * g.po1 + a0 + 4 * lg, g.po1 * g.po1);
  };
  float sc5 = 1.f;  // FP16: one scale for the item's T
  if (H::kScaled) sc5 = pow2_scale(__builtin_bit_cast(float, tmax[blockIdx.y]));
  load_b(0);
  issue(sb, 0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    const float* __restrict__ cur = sb + (c & 1) * celems;
    const int a0 = c * kc;
    const Split4 be = be_n, bo = bo_n;
    if (c + 1 < nchunks) {
      load_b(a0 + kc);
      issue(sb + ((c + 1) & 1) * celems, a0 + kc);
    }
    si_k_step<H, NT, NTO>(acc1, cur + 4 * lg * p2 + li, p2, pe2, be, sc5);
    if (has_o && a0 < g.po1)
      si_k_step<H, NT, NTO>(acc1 + 2 * NT, cur + (kc + 4 * lg) * p2 + li, p2, pe2, bo, sc5);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  // split the W tiles once; they are the B operands of every y' tile
  // (FP16: acc1 carries 2^12 sc5 and is rescaled per wave)
  float m6 = 1.f, un6 = 1.f;
  if (H::kScaled) {
    const float un5 = 1.f / (H::kVScale * sc5);
    const float sc6 = pow2_scale(tiles_absmax<4 * NT>(acc1) * un5);
    m6 = un5 * sc6;
    un6 = 1.f / (H::kVScale * sc6);
  }
  Split4 bs[4 * NT];
#pragma unroll
  for (int k = 0; k < 4 * NT; ++k)
    bs[k] = split4<H>(acc1[k][0], acc1[k][1], acc1[k][2], acc1[k][3], m6);

  const bool xin = zin && xp < g.me1;
  const long long zoff = (long long)(zin ? z : 0) * g.n1 * g.n2;
  const Item item = items[it];
  const S* __restrict__ pi = psi + (long long)item.i * g.N + zoff;
  const S* __restrict__ pj = psi + (long long)(MODE == 1 ? item.j : item.i) * g.N + zoff;
  S* __restrict__ vj = dst + (long long)(MODE == 1 ? item.j : item.i) * g.N + zoff;
  S* __restrict__ vi = dst + (long long)item.i * g.N + zoff;
  const bool offdiag = MODE == 1 && item.i != item.j;
  const float oi = MODE == 1 ? (float)occ[item.i] : 0.f;
  const float oj = MODE == 1 ? (float)occ[item.j] : 0.f;
  // phi of this slab into LDS (the staged chunks are no longer read), then
  // the plane's rows through the update
  float* __restrict__ plane = sb;
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    f4 Q[4];
    const short* VE2 = VL ? vE : e.E[1];
    const short* VO2 = VL ? vO : e.O[1];
    const int lde = VL ? sinv_ld(pe2) : pe2, ldo = VL ? sinv_ld(po2) : po2;
    if (has_o)
      si_mode2<H, NT, NTO, true>(bs, Q, u, VE2, VO2, lde, ldo, pe2 * lde, po2 * ldo, lg, li);
    else
      si_mode2<H, NT, NTO, false>(bs, Q, u, VE2, VO2, lde, ldo, pe2 * lde, po2 * ldo, lg, li);
    if (H::kScaled) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int r = 0; r < 4; ++r) Q[k][r] *= un6;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float ee = Q[0][r], eo = has_o ? Q[1][r] : 0.f;
      const float oe = u < NTO ? Q[2][r] : 0.f, oo = (has_o && u < NTO) ? Q[3][r] : 0.f;
      const float ph[4] = {ee + eo + oe + oo, ee - eo + oe - oo, ee + eo - oe - oo,
                           ee - eo - oe + oo};
      plane_put(plane, g, xin, xp, kTile * u + 4 * lg + r, ph);
    }
  }
  __syncthreads();
  if (!zin) return;
  // FP32 update (Vx psi is accumulated in FP32 on this path)
  rows_apply<float, S, MODE, 4>(plane, g, plane_rows(g), tid - s * nstr * 64, nstr * 64, pi, pj,
                                vj, vi, oi, oj, offdiag);
}

template <class K>
void allow_lds(K kernel, size_t lds) {
  allow_dynamic_lds((const void*)kernel, lds);
}

#define KX_NT_CASES(MACRO) MACRO(1) MACRO(2) MACRO(3) MACRO(4) MACRO(5)

template <class H, class S>
hipError_t sfwd_launch(int mode, const Geom& g, const SlabPlan& p, const EigS& e, const S* src,
                       const Item* items, int nitems, float* T, const float* omax,
                       hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  const dim3 grid((g.n3 + p.slabs - 1) / p.slabs, nitems, p.qsplit);
  const dim3 block(64 * p.waves);
  const size_t lb = p.lds_bytes;
  const bool of = g.po1 == g.pe1;
  const int wps = (p.qsplit == 1 ? 2 : 1) * (g.p2 / kTile);
  const bool xst = p.kc * g.pe1 > kFwdPos * wps * 64;
  switch (g.pe1 / kTile) {
#define KX_CASE(NT)                                                                          \
  case NT: {                                                                                 \
    constexpr int MT = fwd_mt(NT);                                                           \
    auto k = xst ? (mode == 1 ? (of ? split_forward<H, S, NT, true, 1, true, MT>                  \
                                    : split_forward<H, S, NT, false, 1, true, MT>)                \
                              : (of ? split_forward<H, S, NT, true, 0, true, MT>                  \
                                    : split_forward<H, S, NT, false, 0, true, MT>))               \
                 : (mode == 1 ? (of ? split_forward<H, S, NT, true, 1, false, MT>                 \
                                    : split_forward<H, S, NT, false, 1, false, MT>)               \
                              : (of ? split_forward<H, S, NT, true, 0, false, MT>                 \
                                    : split_forward<H, S, NT, false, 0, false, MT>));             \
    allow_lds(k, lb);                                                                        \
    hipLaunchKernelGGL(k, grid, block, lb, st, g, e, src, items, T, p.slabs, p.kc, p.qsplit, \
                       omax);                                                                \
    break;                                                                                   \
  }
    KX_NT_CASES(KX_CASE)
#undef KX_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class H>
hipError_t spen_launch(const Geom& g, const PencilPlan& p, const EigS& e, const double* F,
                       int nitems, float* T, double* epart, unsigned* tmax, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  const long long nstrips = g.slab / kTile;
  const int w = p.waves;
  const dim3 grid((unsigned)((nstrips + w - 1) / w), nitems);
  const dim3 block(64 * w);
  const bool of = g.po3 == g.pe3;
  const size_t lb = p.lds_bytes;
  if (lb > 0 && lb < spen_vbytes(g)) return hipErrorInvalidValue;
  switch (g.pe3 / kTile) {
#define KX_CASE(NT)                                                                      \
  case NT: {                                                                             \
    constexpr int MT = pen_mt(NT);                                                       \
    auto k = lb > 0 ? (of ? split_pencil<H, NT, true, true, MT>                          \
                          : split_pencil<H, NT, false, true, MT>)                        \
                    : (of ? split_pencil<H, NT, true, false, MT>                         \
                          : split_pencil<H, NT, false, false, MT>);                      \
    allow_lds(k, lb);                                                                    \
    hipLaunchKernelGGL(k, grid, block, lb, st, g, e, F, T, epart, tmax);                 \
    break;                                                                               \
  }
    KX_NT_CASES(KX_CASE)
#undef KX_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class H, class S>
hipError_t sinv_launch(int mode, const Geom& g, const SlabPlan& p, const EigS& e, const float* T,
                       const Item* items, int nitems, const S* psi, const double* occ, S* dst,
                       const unsigned* tmax, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  if (p.kc != kTile) return hipErrorInvalidValue;  // chunks are exactly one k-step
  const dim3 grid((g.n3 + p.slabs - 1) / p.slabs, nitems);
  const dim3 block(64 * p.waves);
  const size_t lb = p.lds_bytes;
  const bool of = g.po2 == g.pe2;
  switch (g.pe2 / kTile) {
#define KX_CASE(NT)                                                                         \
  case NT: {                                                                                \
    constexpr int MT = inv_mt(NT);                                                          \
    auto k = mode == 1 ? (of ? split_inverse<H, S, NT, true, 1, false, MT> : split_inverse<H, S, NT, false, 1, false, MT>) \
                       : (of ? split_inverse<H, S, NT, true, 0, false, MT> : split_inverse<H, S, NT, false, 0, false, MT>); \
    if (p.vlds)                                                                             \
      k = mode == 1 ? (of ? split_inverse<H, S, NT, true, 1, true, MT> : split_inverse<H, S, NT, false, 1, true, MT>) \
                    : (of ? split_inverse<H, S, NT, true, 0, true, MT> : split_inverse<H, S, NT, false, 0, true, MT>); \
    allow_lds(k, lb);                                                                       \
    hipLaunchKernelGGL(k, grid, block, lb, st, g, e, T, items, psi, occ, dst, p.slabs, p.kc, \
                       tmax);                                                               \
    break;                                                                                  \
  }
    KX_NT_CASES(KX_CASE)
#undef KX_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

Plan make_split_plan(const Geom& g, size_t max_lds) {
  // Same workgroup shapes as the FP32 path; chunks of exactly one k-step and
  // no V blocks in LDS (the pre-split blocks are read through the caches).
  Plan pl = make_plan(g, max_lds, sizeof(float));
  // staging beyond the per-thread register budget falls back to direct
  // loads in these kernels, so every shape is accepted
  SlabPlan& f = pl.fwd;
  f.kc = kSplitKc;
  f.vlds = false;
  f.ok = true;
  const int wrow = f.qsplit == 1 ? g.p1 : g.pe1;
  f.lds_bytes = (size_t)f.slabs * 2 * 2 * f.kc * wrow * sizeof(float);
  SlabPlan& v = pl.inv;
  v.kc = kSplitKc;
  v.vlds = false;
  v.ok = true;
  v.lds_bytes = split_inv_lds(g, v.slabs, false);
  pl.pen.lds_bytes = 0;
  return pl;
}

hipError_t launch_forward_s(int storage, int mode, const Geom& g, const SlabPlan& p,
                            const EigS& e, const void* src, const Item* items, int nitems,
                            float* T, hipStream_t s, const SplitAux& aux) {
  if (aux.h16 && !aux.omax) return hipErrorInvalidValue;
  if (storage == KX_F64)
    return aux.h16 ? sfwd_launch<F16, double>(mode, g, p, e, (const double*)src, items, nitems, T,
                                              aux.omax, s)
                   : sfwd_launch<BF16, double>(mode, g, p, e, (const double*)src, items, nitems,
                                               T, nullptr, s);
  return aux.h16 ? sfwd_launch<F16, float>(mode, g, p, e, (const float*)src, items, nitems, T,
                                           aux.omax, s)
                 : sfwd_launch<BF16, float>(mode, g, p, e, (const float*)src, items, nitems, T,
                                            nullptr, s);
}

hipError_t launch_pencil_s(const Geom& g, const PencilPlan& p, const EigS& e, const double* F,
                           int nitems, float* T, double* epart, hipStream_t s,
                           const SplitAux& aux) {
  if (aux.h16 && !aux.tmax) return hipErrorInvalidValue;
  return aux.h16 ? spen_launch<F16>(g, p, e, F, nitems, T, epart, aux.tmax, s)
                 : spen_launch<BF16>(g, p, e, F, nitems, T, epart, nullptr, s);
}

hipError_t launch_inverse_s(int storage, int mode, const Geom& g, const SlabPlan& p,
                            const EigS& e, const float* T, const Item* items, int nitems,
                            const void* psi, const double* occ, void* dst, hipStream_t s,
                            const SplitAux& aux) {
  if (aux.h16 && !aux.tmax) return hipErrorInvalidValue;
  if (storage == KX_F64)
    return aux.h16 ? sinv_launch<F16, double>(mode, g, p, e, T, items, nitems,
                                              (const double*)psi, occ, (double*)dst, aux.tmax, s)
                   : sinv_launch<BF16, double>(mode, g, p, e, T, items, nitems,
                                               (const double*)psi, occ, (double*)dst, nullptr, s);
  return aux.h16 ? sinv_launch<F16, float>(mode, g, p, e, T, items, nitems, (const float*)psi,
                                           occ, (float*)dst, aux.tmax, s)
                 : sinv_launch<BF16, float>(mode, g, p, e, T, items, nitems, (const float*)psi,
                                            occ, (float*)dst, nullptr, s);
}

namespace {
__global__ void __launch_bounds__(256) absmax_kernel(const void* x, int f64, long long n, float* out) {
  // one workgroup per vector
  const long long base = (long long)blockIdx.x * n;
  float m = 0.f;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) {
    const float v = f64 ? (float)fabs(((const double*)x)[base + i]) : fabsf(((const float*)x)[base + i]);
    m = fmaxf(m, v);
  }
  m = wave_max(m);
  __shared__ float red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}
}  // namespace

hipError_t launch_absmax(const void* x, int storage, long long n, int count, float* out,
                         hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(absmax_kernel, dim3(count), dim3(256), 0, s, x, storage == KX_F64 ? 1 : 0, n,
                     out);
  return hipGetLastError();
}

}  // namespace kx
