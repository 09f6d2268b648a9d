// Internal declarations of auxiliary kernels outside the transform passes
// (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "kx_internal.h"

namespace kx {

// The compressed exchange of complex fields runs the real algebra on their
// real form: a complex field of N values, interleaved (re, im), is a real
// vector of 2 N values, and the real form of the span of n complex fields is
// spanned by the 2 n real vectors {z_j, i z_j}.  dst (2 n vectors of 2 N
// doubles) = [src_0 .. src_{n-1}, i src_0 .. i src_{n-1}].
hipError_t launch_realify(const double* src, int n, long long N, double* dst, hipStream_t s);

}  // namespace kx

namespace kx {

// ---- the two-stage FP64 exchange (kx_accum.hip).  The pairs i <= j of norb
// orbitals are taken in tiles of kXTile x kXTile orbitals: rows i in block a,
// columns j in block b >= a, tiles in row-major order of the block triangle,
// the pairs of a tile in row-major order.  The inverse pass writes the
// tile's potentials phi_ij, and one kernel applies them to Vx psi, reading
// and writing each of the tile's orbitals once.
constexpr int kXTile = 8;
constexpr int kXTileMaxOrb = 4096;  // larger orbital counts keep the fused inverse pass
// orbitals in block a
__host__ __device__ inline int xtile_size(int a, int norb) {
  const int r = norb - kXTile * a;
  return r < kXTile ? r : kXTile;
}
// pairs of the tile (a, b), b >= a
__host__ __device__ inline int xtile_pairs(int a, int b, int norb) {
  const int sa = xtile_size(a, norb);
  return a == b ? sa * (sa + 1) / 2 : sa * xtile_size(b, norb);
}
// the items of every tile, in order (norb(norb+1)/2 items)
hipError_t launch_tile_schedule(int norb, Item* out, hipStream_t s);
// Vx psi -= the tile (a, b)'s pairs: phi holds its pairs' potentials
// (field t for the tile's pair t, storage phi_storage); psi, vx of storage
// KX_F64 / KX_F32
hipError_t launch_tile_accumulate(int storage, int phi_storage, const void* phi, int a, int b,
                                  int norb, long long N, const void* psi, const double* occ,
                                  void* vx, hipStream_t s);

}  // namespace kx
