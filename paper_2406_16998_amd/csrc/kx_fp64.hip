// FP64 transform kernels for X = f(L) B (Sec. III, Eqs. (20)-(21)) and the
// exchange operator built on it (Sec. II, Eqs. (3)-(5)).
//
// Three passes per batch of independent items (an item is one field for
// apply_fL, or one orbital pair (i, j) for the exchange):
//
//   forward   per (item, z-slab, 16-wide b strip):
//               S = rho[z]  (or psi_i[z] * psi_j[z])            (pair product)
//               T'[x][b] = sum_y S[y][x] V2[y][b]               (mode 2)
//               T1[a][b] = sum_x V1[x][a] T'[x][b]              (mode 1)
//   pencil    per (item, 16 columns q = (a, b)):
//               B~[c][q] = sum_z V3[z][c] T1[z][q]              (mode 3)
//               e += F[c][q] B~^2;  X~ = F B~                    (Hadamard, Eq. (21b))
//               T2[z][q] = sum_c V3[z][c] X~[c][q]              (mode 3 inverse)
//   inverse   per (item, z-slab, 16-wide x strip):
//               W[b][x] = sum_a T2[a][b] V1[x][a]               (mode 1 inverse)
//               phi[y][x] = sum_b V2[y][b] W[b][x]              (mode 2 inverse)
//               phi -> output, or (Vx psi)_j -= occ_i phi psi_i and,
//               for i != j, (Vx psi)_i -= occ_j phi psi_j        (Eq. (3))
//
// Every contraction runs on v_mfma_f64_16x16x4f64.  Operand layout of that
// instruction on gfx950 (lane l = 0..63, li = l % 16, lg = l / 16; measured):
//   A (16 x 4):  lane l holds A[li][lg]
//   B (4 x 16):  lane l holds B[lg][li]
//   D (16 x 16): lane l, element r holds D[4*r + lg][li]
// So element r of an accumulator tile t is, lane for lane, the B operand of
// the k-step that covers k = 16 t + 4 r .. 16 t + 4 r + 3.  The second product
// of each pass consumes the first one's accumulators directly as B operands:
// the intermediate of the first product never leaves registers.
//
// Intermediate layout (our own): T[item][z][a][b], a < p1, b < p2 (padded to
// 16, zero padding), z < p3; V_k and their transposes are zero-padded too.
#include <hip/hip_runtime.h>

#include "kx_internal.h"

namespace kx {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dbl4 mfma_f64(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- forward
template <int NT1, int MODE>
__global__ void __launch_bounds__(64)
forward_kernel(Geom g, Eig e, const double* __restrict__ src, const Item* __restrict__ items,
               double* __restrict__ T) {
  const int lane = threadIdx.x;
  const int li = lane & 15, lg = lane >> 4;
  const int b0 = blockIdx.x * kTile;
  const int z = blockIdx.y;
  const int it = blockIdx.z;
  const Item item = items[it];
  const long long zoff = (long long)z * g.n1 * g.n2;
  const double* __restrict__ s0 = src + (long long)item.i * g.N + zoff;
  const double* __restrict__ s1 = src + (long long)(MODE == 1 ? item.j : item.i) * g.N + zoff;
  const double* __restrict__ V1 = e.V[0];
  const double* __restrict__ V2 = e.V[1];

  dbl4 acc1[NT1];
#pragma unroll
  for (int t = 0; t < NT1; ++t) acc1[t] = dbl4{0.0, 0.0, 0.0, 0.0};

  // mode 2:  C[x][b] += A[x][y] B[y][b],  A = S^T, B = V2
  for (int y0 = 0; y0 < g.n2; y0 += 4) {
    const int y = y0 + lg;
    const double bop = V2[y * g.p2 + b0 + li];
    const bool yin = y < g.n2;
#pragma unroll
    for (int t = 0; t < NT1; ++t) {
      const int x = kTile * t + li;
      double a = 0.0;
      if (yin && x < g.n1) {
        a = s0[y * g.n1 + x];
        if (MODE == 1) a *= s1[y * g.n1 + x];
      }
      acc1[t] = mfma_f64(a, bop, acc1[t]);
    }
  }

  // mode 1:  C[a][b] += A[a][x] B[x][b],  A = V1^T, B = T' (registers)
  dbl4 acc2[NT1];
#pragma unroll
  for (int u = 0; u < NT1; ++u) acc2[u] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < NT1; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int x = kTile * t + 4 * r + lg;
      const double bop = acc1[t][r];
      const double* __restrict__ vrow = V1 + x * g.p1 + li;
#pragma unroll
      for (int u = 0; u < NT1; ++u) acc2[u] = mfma_f64(vrow[kTile * u], bop, acc2[u]);
    }
  }

  double* __restrict__ Tz = T + (long long)it * g.slot + (long long)z * g.slab;
#pragma unroll
  for (int u = 0; u < NT1; ++u) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = kTile * u + 4 * r + lg;
      Tz[a * g.p2 + b0 + li] = acc2[u][r];
    }
  }
}

// ---------------------------------------------------------------- pencil
template <int NT3>
__global__ void __launch_bounds__(64)
pencil_kernel(Geom g, Eig e, const double* __restrict__ F, double* __restrict__ T,
              double* __restrict__ epart) {
  const int lane = threadIdx.x;
  const int li = lane & 15, lg = lane >> 4;
  const long long q0 = (long long)blockIdx.x * kTile;
  const int it = blockIdx.y;
  double* __restrict__ Tb = T + (long long)it * g.slot;
  const double* __restrict__ V3 = e.V[2];
  const double* __restrict__ V3T = e.VT[2];

  dbl4 acc[NT3];
#pragma unroll
  for (int t = 0; t < NT3; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
  // mode 3:  C[c][q] += A[c][z] B[z][q],  A = V3^T, B = T1
  for (int z0 = 0; z0 < g.n3; z0 += 4) {
    const int z = z0 + lg;
    const double bop = (z < g.n3) ? Tb[z * g.slab + q0 + li] : 0.0;
    const double* __restrict__ vrow = V3 + z * g.p3 + li;
#pragma unroll
    for (int t = 0; t < NT3; ++t) acc[t] = mfma_f64(vrow[kTile * t], bop, acc[t]);
  }

  // Hadamard product with f(Lambda) and the pair-energy partial sum F B~^2
  double esum = 0.0;
#pragma unroll
  for (int t = 0; t < NT3; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = kTile * t + 4 * r + lg;
      const double f = F[c * g.slab + q0 + li];
      const double v = acc[t][r];
      esum += f * v * v;
      acc[t][r] = f * v;
    }
  }

  // inverse mode 3:  C[z][q] += A[z][c] B[c][q],  A = V3, B = X~ (registers)
  dbl4 out[NT3];
#pragma unroll
  for (int u = 0; u < NT3; ++u) out[u] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < NT3; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = kTile * t + 4 * r + lg;
      const double bop = acc[t][r];
      const double* __restrict__ vrow = V3T + c * g.p3 + li;
#pragma unroll
      for (int u = 0; u < NT3; ++u) out[u] = mfma_f64(vrow[kTile * u], bop, out[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < NT3; ++u) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int z = kTile * u + 4 * r + lg;
      if (z < g.n3) Tb[z * g.slab + q0 + li] = out[u][r];
    }
  }

  // fixed-order wave reduction of the energy partial
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) esum += __shfl_xor(esum, o);
  if (epart != nullptr && lane == 0) epart[(long long)it * gridDim.x + blockIdx.x] = esum;
}

// ---------------------------------------------------------------- inverse
template <int NT2, int MODE>
__global__ void __launch_bounds__(64)
inverse_kernel(Geom g, Eig e, const double* __restrict__ T, const Item* __restrict__ items,
               const double* __restrict__ psi, const double* __restrict__ occ,
               double* __restrict__ dst) {
  const int lane = threadIdx.x;
  const int li = lane & 15, lg = lane >> 4;
  const int x0 = blockIdx.x * kTile;
  const int z = blockIdx.y;
  const int it = blockIdx.z;
  const double* __restrict__ Tz = T + (long long)it * g.slot + (long long)z * g.slab;
  const double* __restrict__ V1T = e.VT[0];
  const double* __restrict__ V2T = e.VT[1];

  dbl4 acc1[NT2];
#pragma unroll
  for (int t = 0; t < NT2; ++t) acc1[t] = dbl4{0.0, 0.0, 0.0, 0.0};
  // inverse mode 1:  C[b][x] += A[b][a] B[a][x],  A = T2^T, B = V1^T
  for (int a0 = 0; a0 < g.n1; a0 += 4) {
    const int a = a0 + lg;
    const double bop = V1T[a * g.p1 + x0 + li];
    const double* __restrict__ trow = Tz + a * g.p2 + li;
#pragma unroll
    for (int t = 0; t < NT2; ++t) acc1[t] = mfma_f64(trow[kTile * t], bop, acc1[t]);
  }

  // inverse mode 2:  C[y][x] += A[y][b] B[b][x],  A = V2, B = W (registers)
  dbl4 acc2[NT2];
#pragma unroll
  for (int u = 0; u < NT2; ++u) acc2[u] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < NT2; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int b = kTile * t + 4 * r + lg;
      const double bop = acc1[t][r];
      const double* __restrict__ vrow = V2T + b * g.p2 + li;
#pragma unroll
      for (int u = 0; u < NT2; ++u) acc2[u] = mfma_f64(vrow[kTile * u], bop, acc2[u]);
    }
  }

  const int x = x0 + li;
  if (x >= g.n1) return;
  const long long zoff = (long long)z * g.n1 * g.n2 + x;
  if (MODE == 0) {
    double* __restrict__ out = dst + (long long)items[it].i * g.N + zoff;
#pragma unroll
    for (int u = 0; u < NT2; ++u) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int y = kTile * u + 4 * r + lg;
        if (y < g.n2) out[y * g.n1] = acc2[u][r];
      }
    }
  } else {
    const Item item = items[it];
    const double oi = occ[item.i], oj = occ[item.j];
    const double* __restrict__ pi = psi + (long long)item.i * g.N + zoff;
    const double* __restrict__ pj = psi + (long long)item.j * g.N + zoff;
    double* __restrict__ vj = dst + (long long)item.j * g.N + zoff;
    double* __restrict__ vi = dst + (long long)item.i * g.N + zoff;
    const bool offdiag = item.i != item.j;
#pragma unroll
    for (int u = 0; u < NT2; ++u) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int y = kTile * u + 4 * r + lg;
        if (y < g.n2) {
          const long long o = (long long)y * g.n1;
          const double phi = acc2[u][r];
          vj[o] -= (oi * phi) * pi[o];
          if (offdiag) vi[o] -= (oj * phi) * pj[o];
        }
      }
    }
  }
}

// ---------------------------------------------------------------- energies
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

}  // namespace

#define KX_NT_CASES(MACRO) \
  MACRO(1) MACRO(2) MACRO(3) MACRO(4) MACRO(5) MACRO(6) MACRO(7) MACRO(8) MACRO(9) MACRO(10)

hipError_t launch_forward_f64(int mode, const Geom& g, const Eig& e, const double* src,
                              const Item* items, int nitems, double* T, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  const dim3 grid(g.p2 / kTile, g.n3, nitems);
  const int nt = g.p1 / kTile;
  switch (nt) {
#define KX_CASE(NT)                                                                        \
  case NT:                                                                                 \
    if (mode == 1)                                                                         \
      hipLaunchKernelGGL((forward_kernel<NT, 1>), grid, dim3(64), 0, s, g, e, src, items, T); \
    else                                                                                   \
      hipLaunchKernelGGL((forward_kernel<NT, 0>), grid, dim3(64), 0, s, g, e, src, items, T); \
    break;
    KX_NT_CASES(KX_CASE)
#undef KX_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pencil_f64(const Geom& g, const Eig& e, const double* F, int nitems, double* T,
                             double* epart, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  const dim3 grid((unsigned)(g.slab / kTile), nitems);
  const int nt = g.p3 / kTile;
  switch (nt) {
#define KX_CASE(NT)                                                                         \
  case NT:                                                                                  \
    hipLaunchKernelGGL((pencil_kernel<NT>), grid, dim3(64), 0, s, g, e, F, T, epart); \
    break;
    KX_NT_CASES(KX_CASE)
#undef KX_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_inverse_f64(int mode, const Geom& g, const Eig& e, const double* T,
                              const Item* items, int nitems, const double* psi, const double* occ,
                              double* dst, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  const dim3 grid(g.p1 / kTile, g.n3, nitems);
  const int nt = g.p2 / kTile;
  switch (nt) {
#define KX_CASE(NT)                                                                          \
  case NT:                                                                                   \
    if (mode == 1)                                                                           \
      hipLaunchKernelGGL((inverse_kernel<NT, 1>), grid, dim3(64), 0, s, g, e, T, items, psi, \
                         occ, dst);                                                          \
    else                                                                                     \
      hipLaunchKernelGGL((inverse_kernel<NT, 0>), grid, dim3(64), 0, s, g, e, T, items, psi, \
                         occ, dst);                                                          \
    break;
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
