// The two-stage exchange: the inverse pass writes the potentials phi_ij of
// one tile of orbital pairs (FP64, or FP32 in the reduced precisions), and
// the kernels here apply the tile to
// Vx psi (Sec. II, the exchange operator in Poisson form):
//   (Vx psi)_j -= occ_i phi_ij psi_i,   (Vx psi)_i -= occ_j phi_ij psi_j (i != j).
// A thread owns one grid point and holds the tile's orbitals (psi and the
// Vx psi being accumulated) in registers, so each orbital is read and
// written once per tile instead of once per pair.
#include <hip/hip_runtime.h>

#include "kx_aux.h"
#include "kx_internal.h"

namespace kx {
namespace {

// tile tau of the row-major triangle of nbk blocks -> (a, b)
__device__ __forceinline__ void xtile_of(int tau, int nbk, int& a, int& b) {
  a = 0;
  int first = 0;  // index of tile (a, a)
  while (first + (nbk - a) <= tau) {
    first += nbk - a;
    ++a;
  }
  b = a + (tau - first);
}

// one thread per tile: the tile's items at its offset (all earlier tiles' pairs)
__global__ void tile_schedule_kernel(int norb, Item* __restrict__ out) {
  const int nbk = (norb + kXTile - 1) / kXTile;
  const int ntiles = nbk * (nbk + 1) / 2;
  const int tau = blockIdx.x * blockDim.x + threadIdx.x;
  if (tau >= ntiles) return;
  int a, b;
  xtile_of(tau, nbk, a, b);
  long long off = 0;
  for (int a2 = 0; a2 < a; ++a2)
    for (int b2 = a2; b2 < nbk; ++b2) off += xtile_pairs(a2, b2, norb);
  for (int b2 = a; b2 < b; ++b2) off += xtile_pairs(a, b2, norb);
  const int sa = xtile_size(a, norb), sb = xtile_size(b, norb);
  for (int r = 0; r < sa; ++r)
    for (int c = 0; c < sb; ++c) {
      const int i = kXTile * a + r, j = kXTile * b + c;
      if (i > j) continue;
      Item it;
      it.i = i;
      it.j = j;
      out[off++] = it;
    }
}

template <class P, class S>
__global__ void __launch_bounds__(256)
tile_accumulate_kernel(const P* __restrict__ phi, int a, int b, int norb, long long N,
                       const S* __restrict__ psi, const double* __restrict__ occ,
                       S* __restrict__ vx) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= N) return;
  const bool diag = a == b;
  const int sa = xtile_size(a, norb), sb = xtile_size(b, norb);
  const int r0 = kXTile * a, c0 = kXTile * b;
  // slots: columns c0 + k in k < kXTile, rows r0 + r in kXTile + r (or, on a
  // diagonal tile, in the columns' slots)
  constexpr int kS = 2 * kXTile;
  double u[kS], w[kS], o[kS];
#pragma unroll
  for (int k = 0; k < kS; ++k) {
    const bool col = k < kXTile;
    const int q = col ? k : k - kXTile;
    const bool live = col ? q < sb : (!diag && q < sa);
    const int orb = col ? c0 + q : r0 + q;
    u[k] = live ? (double)psi[(long long)orb * N + x] : 0.0;
    w[k] = live ? (double)vx[(long long)orb * N + x] : 0.0;
    o[k] = live ? occ[orb] : 0.0;
  }
  int t = 0;
#pragma unroll
  for (int r = 0; r < kXTile; ++r) {
    const int rs = diag ? r : kXTile + r;  // the row's slot
#pragma unroll
    for (int c = 0; c < kXTile; ++c) {
      if (r >= sa || c >= sb || (diag && r > c)) continue;
      const double p = (double)phi[(long long)t * N + x];
      ++t;
      double ur = 0.0, orr = 0.0;
#pragma unroll
      for (int k = 0; k < kS; ++k)
        if (k == rs) {
          ur = u[k];
          orr = o[k];
        }
      w[c] -= orr * p * ur;  // (Vx psi)_j -= occ_i phi_ij psi_i
      if (diag && r == c) continue;
      const double d = o[c] * p * u[c];  // (Vx psi)_i -= occ_j phi_ij psi_j
#pragma unroll
      for (int k = 0; k < kS; ++k)
        if (k == rs) w[k] -= d;
    }
  }
#pragma unroll
  for (int k = 0; k < kS; ++k) {
    const bool col = k < kXTile;
    const int q = col ? k : k - kXTile;
    const bool live = col ? q < sb : (!diag && q < sa);
    if (live) vx[(long long)(col ? c0 + q : r0 + q) * N + x] = (S)w[k];
  }
}

}  // namespace

hipError_t launch_tile_schedule(int norb, Item* out, hipStream_t s) {
  if (norb <= 0) return hipSuccess;
  const int nbk = (norb + kXTile - 1) / kXTile;
  const int ntiles = nbk * (nbk + 1) / 2;
  hipLaunchKernelGGL(tile_schedule_kernel, dim3((ntiles + 255) / 256), dim3(256), 0, s, norb, out);
  return hipGetLastError();
}

hipError_t launch_tile_accumulate(int storage, int phi_storage, const void* phi, int a, int b,
                                  int norb, long long N, const void* psi, const double* occ,
                                  void* vx, hipStream_t s) {
  const dim3 grid((unsigned)((N + 255) / 256));
#define KX_ACC(P, S)                                                                          \
  hipLaunchKernelGGL((tile_accumulate_kernel<P, S>), grid, dim3(256), 0, s, (const P*)phi, a, b, \
                     norb, N, (const S*)psi, occ, (S*)vx)
  if (phi_storage == KX_F64) {
    if (storage == KX_F64)
      KX_ACC(double, double);
    else
      KX_ACC(double, float);
  } else {
    if (storage == KX_F64)
      KX_ACC(float, double);
    else
      KX_ACC(float, float);
  }
#undef KX_ACC
  return hipGetLastError();
}

}  // namespace kx
