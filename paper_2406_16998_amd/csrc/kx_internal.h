// Internal declarations shared by the host API (kx_api.cpp) and the HIP
// kernel translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/kx.h"

namespace kx {

constexpr int kTile = 16;     // MFMA tile edge (v_mfma_f64_16x16x4f64)
constexpr int kMaxN = 160;    // largest supported n_k
constexpr int kMaxNT = kMaxN / kTile;

inline int pad16(int n) { return (n + kTile - 1) / kTile * kTile; }

// Geometry passed by value to every transform kernel.
struct Geom {
  int n1, n2, n3;     // grid points
  int p1, p2, p3;     // padded to multiples of 16
  long long N;        // n1*n2*n3 (field stride in psi / rho / vxpsi)
  long long slab;     // p1*p2  (one z-slab of the intermediate, [a][b])
  long long slot;     // p3*p1*p2 (one intermediate field)
};

// Device copies of the per-axis eigensystems, padded with zeros:
//   V[k]  [i][a] row-major (p_k x p_k), column a = eigenvector a
//   VT[k] [a][i] row-major
//   lam[k] p_k values (zeros beyond n_k)
struct Eig {
  const double* V[3];
  const double* VT[3];
};

// One item of a transform batch: for exchange (i, j) orbital indices; for
// apply_fL (b, -1) with b the field index.
struct Item {
  int i, j;
};

// ---- setup kernels (kx_setup.hip) ----
hipError_t launch_jacobi(double* A, double* V, int n, int max_sweeps, double* lam_pad, double* Vpad,
                         double* VTpad, int np, double* diag_out, hipStream_t s);
hipError_t launch_ftable(const double* lam1, const double* lam2, const double* lam3, const Geom& g,
                         int kernel, double omega, double* F, hipStream_t s);
hipError_t launch_check_orth(const double* V, int n, int np, double* out2, hipStream_t s);

// ---- FP64 transform kernels (kx_fp64.hip) ----
// mode: 0 = apply_fL (rho -> phi), 1 = exchange (psi -> vxpsi)
hipError_t launch_forward_f64(int mode, const Geom& g, const Eig& e, const double* src,
                              const Item* items, int nitems, double* T, hipStream_t s);
hipError_t launch_pencil_f64(const Geom& g, const Eig& e, const double* F, int nitems, double* T,
                             double* epart, hipStream_t s);
hipError_t launch_inverse_f64(int mode, const Geom& g, const Eig& e, const double* T,
                              const Item* items, int nitems, const double* psi, const double* occ,
                              double* dst, hipStream_t s);
// per-item energies: pair_e[idx[k]] = dV * sum_s epart[k*nstrips + s]
hipError_t launch_pair_energy(const double* epart, int nstrips, const Item* items, int nitems,
                              int norb, double dV, double* pair_e, hipStream_t s);
// E_x = -1/4 sum_{i<=j} m_ij occ_i occ_j pair_e, m = 1 (i == j) or 2
hipError_t launch_exchange_energy(const double* pair_e, const double* occ, int norb, double* ex,
                                  hipStream_t s);

__host__ __device__ inline long long pair_index(int i, int j, int norb) {
  // i <= j, row-major upper triangle
  return (long long)i * norb - (long long)i * (i - 1) / 2 + (j - i);
}

}  // namespace kx
