// Internal declarations shared by the host API (kx_api.cpp) and the HIP
// kernel translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/kx.h"

namespace kx {

constexpr int kTile = 16;  // MFMA tile edge (v_mfma_f64_16x16x4f64)
constexpr int kMaxN = 160; // largest supported n_k

inline int pad16(int n) { return (n + kTile - 1) / kTile * kTile; }

// Every 1-D matrix L_k is centrosymmetric (J L_k J = L_k with J the index
// reversal): symmetric Toeplitz for homogeneous Dirichlet ends, symmetric
// circulant for periodic ones.  Its eigenvectors therefore split into even
// (v = J v) and odd (v = -J v) ones, and a product with V_k^T becomes two
// half-size products on the folded vector:
//   x_e[i] = x[i] + x[n-1-i] (i < n/2),  x_e[m] = x[m] for the middle of odd n,
//   x_o[i] = x[i] - x[n-1-i] (i < n/2),
//   (V^T x)_even = VE^T x_e,  (V^T x)_odd = VO^T x_o,
// with VE, VO the upper halves of the even / odd eigenvectors.  The inverse
// product unfolds: p = VE y_e, q = VO y_o, x[i] = p[i] + q[i],
// x[n-1-i] = p[i] - q[i].  Mode indices are stored "parity-blocked": even
// modes a in [0, pe), odd modes at pe + [0, po).
struct Geom {
  int n1, n2, n3;
  int me1, me2, me3;  // even half length: ceil(n/2)
  int mo1, mo2, mo3;  // odd half length: floor(n/2)
  int pe1, pe2, pe3;  // pad16(me)
  int po1, po2, po3;  // pad16(mo)
  int p1, p2, p3;     // pe + po: blocked mode-index extent
  long long N;        // n1*n2*n3 (field stride in psi / rho / vxpsi)
  long long slab;     // p1*p2: one z-slab of the intermediate, [a][b] blocked
  long long slot;     // n3*slab: one intermediate field, [z][a][b]
  long long fsize;    // p3*slab: the f table, [c][a][b]
};

// Device copies of the half eigenvector blocks, zero padded, in the operand
// type R of the mode products:
//   VE[k] [i][a] row-major pe_k x pe_k (i < me_k spatial, a < me_k mode)
//   VO[k] [i][a] row-major po_k x po_k
//   VET, VOT their transposes.
template <class R>
struct EigR {
  const R* VE[3];
  const R* VO[3];
  const R* VET[3];
  const R* VOT[3];
};

// Pre-split copies of the same blocks for the split-BF16 products: each is
// three bf16 planes (bit patterns) of pe_k x pe_k (po_k x po_k) elements,
// plane s at offset s * pe_k^2, with V ~ plane0 + plane1 + plane2.
//   E[k] = split(VE[k]) [i][a],  O[k] = split(VO[k]),
//   ET[k] = split(VET[k]) [a][i], OT[k] = split(VOT[k]).
struct EigS {
  const short* E[3];
  const short* O[3];
  const short* ET[3];
  const short* OT[3];
};

// Staging budgets of the slab kernels and their launch bounds (threads per
// workgroup) by register tile count NT, shared by kernels and planner.
constexpr int kFwdPos = 2;  // folded positions staged per thread per chunk (register staging)
// Largest chunk (folded rows) of the forward pass: FP64 operands stage raw
// rows through LDS, FP32 operands through registers.
constexpr int fwd_max_kc(size_t esize) { return esize == 8 ? 8 : 16; }
constexpr int fwd_mt(int nt) { return nt <= 3 ? 1024 : (nt == 4 ? 768 : 640); }
// waves per SIMD the forward pass keeps its registers for: six lets two
// 12-wave workgroups share a CU, so one workgroup's loads overlap the
// other's products
constexpr int fwd_min_waves(int nt) { return nt <= 3 ? 6 : 1; }
constexpr int inv_mt(int nt) { return nt <= 2 ? 1024 : (nt == 3 ? 768 : 512); }
// the FP64 inverse pass with the b parities on separate waves (inverse_bsplit):
// selected by waves = 2 * (pe1 / 16) * slabs
constexpr int inv_bsplit_mt(int nt) { return nt <= 3 ? 768 : 640; }
constexpr int pen_mt(int nt) { return nt <= 2 ? 1024 : 512; }
constexpr int pen_min_waves(int nt) { return nt <= 3 ? 3 : 1; }

// Split inverse pass with its V2 blocks in LDS: row stride (bf16 elements) of
// a staged block, padded by 4 so that the 16 rows of an operand read start in
// different banks, and the bytes of the three planes of both blocks.
__host__ __device__ inline int sinv_ld(int n) { return n + 4; }
__host__ __device__ inline size_t sinv_vbytes(const Geom& g) {
  const size_t b = 2 * 3 * ((size_t)g.pe2 * sinv_ld(g.pe2) + (size_t)g.po2 * sinv_ld(g.po2));
  return (b + 15) / 16 * 16;
}
// Split pencil with its V3 blocks in LDS: row padding (bf16 elements) and the
// bytes of the three planes of both blocks in both orientations.
__host__ __device__ inline int spen_pad() { return 4; }
__host__ __device__ inline size_t spen_vbytes(const Geom& g) {
  return (size_t)2 * 3 * 2 *
         ((size_t)g.pe3 * (g.pe3 + spen_pad()) + (size_t)g.po3 * (g.po3 + spen_pad()));
}
// Elements (of the operand type) of LDS per z-slab of an inverse launch: two
// staged chunks of kc rows, reused afterwards for the output: the slab's phi
// plane (n1 x n2), or one output band (2 kTile rows of n1) at a time.
__host__ __device__ inline size_t inv_slab_elems(const Geom& g, int kc, bool band) {
  const size_t stage = (size_t)2 * 2 * kc * g.p2;
  const size_t out = band ? (size_t)2 * kTile * g.n1 : (size_t)g.n1 * g.n2;
  return ((stage > out ? stage : out) + 3) / 4 * 4;
}
// FP64 / FP32 forward pass, per z-slab: bytes of LDS for one staged range of
// raw rows (kc grid rows of n1 stored values of ssize bytes, in whole 1 KB
// copy segments), and for the slab's two folded buffers ([2][kc][wrow]
// operands of esize bytes) plus, with FP64 operands, two raw stages of four
// ranges.
__host__ __device__ inline int fwd_raw_range(const Geom& g, int kc, size_t ssize) {
  return (int)(((size_t)kc * g.n1 * ssize + 1023) / 1024 * 1024);
}
__host__ __device__ inline size_t fwd_slab_bytes(const Geom& g, int kc, int wrow, size_t esize,
                                                 size_t ssize = 8) {
  return (size_t)2 * 2 * kc * wrow * esize +
         (esize == 8 ? (size_t)2 * 4 * fwd_raw_range(g, kc, ssize) : 0);
}

// Staged rows per chunk of the inverse pass (the chunks are copied to LDS in
// 1 KB segments: 64 bytes per column).
constexpr int inv_kc(size_t esize) { return (int)(64 / esize); }
// Inverse kernels with FP64 operands stream bands, the others whole planes.
__host__ __device__ inline bool inv_band(size_t esize) { return esize == 8; }
// LDS of a split inverse launch, plus the V2 blocks when they are resident.
inline size_t split_inv_lds(const Geom& g, int slabs, bool vlds) {
  return (size_t)slabs * inv_slab_elems(g, kTile, false) * sizeof(float) +
         (vlds ? sinv_vbytes(g) : 0);
}

// One item of a transform batch: an orbital pair (i, j) for the exchange,
// (b, -1) with b the field index for apply_fL.
struct Item {
  int i, j;
};

// Launch shapes, chosen once per grid from the LDS size.
struct SlabPlan {
  int slabs = 1;      // z-slabs per workgroup
  int kc = 8;         // folded K rows staged per chunk
  int waves = 1;      // waves per workgroup
  int qsplit = 1;     // forward: 2 = one x-parity per workgroup
  bool vlds = false;  // the second product's V blocks resident in LDS
  size_t lds_bytes = 0;
  bool ok = true;     // false: the grid's shape does not fit these kernels
};
struct PencilPlan {
  int waves = 8;
  size_t lds_bytes = 0;  // 0: V3 blocks read from global memory
  int per = 0;           // > 0: pipelined kernel, `per` items per wave (tiles <= kPipeMaxNT)
};
constexpr int kPipeMaxNT = 3;  // the pipelined pencil's register budget (two waves per SIMD)
struct Plan {
  SlabPlan fwd, inv;
  PencilPlan pen;
};
// esize: bytes per element of the mode-product operands (8 or 4)
Plan make_plan(const Geom& g, size_t max_lds, size_t esize);
// every valid launch shape (kind 0: double operands, 1: float, 2: split-BF16);
// ssize: bytes of the stored orbitals the shapes are sized for (forward LDS;
// every shape also fits 8-byte storage, for which the launch enlarges it)
void plan_candidates(const Geom& g, size_t max_lds, int kind, std::vector<SlabPlan>& fwd,
                     std::vector<PencilPlan>& pen, std::vector<SlabPlan>& inv,
                     size_t ssize = 8);

// ---- set-up kernels (kx_setup.hip) ----
// Jacobi eigensolver of the symmetric n x n matrix A (global memory); writes
// eigenvalues ascending into lam_pad[0..n) and the eigenvectors, row i
// scaled by rs except row keep_row, into Vpad[i*np + a] and VTpad[a*np + i].
hipError_t launch_jacobi(double* A, double* V, int n, int max_sweeps, double rs, int keep_row,
                         double* lam_pad, double* Vpad, double* VTpad, int np, double* diag_out,
                         hipStream_t s);
// f of the summed eigenvalues in the blocked [c][a][b] order, zero on padding
// zero: for KX_KERNEL_COULOMB with zero.on, every eigenvalue sum lam <= zero.tol
// (the zero mode) takes the value zero.val instead of 4 pi / lam
struct ZeroMode {
  int on = 0;
  double val = 0.0, tol = 0.0;
};
hipError_t launch_ftable(const double* const lamE[3], const double* const lamO[3], const Geom& g,
                         int kernel, double omega, double* F, hipStream_t s,
                         const ZeroMode& zero = ZeroMode());

// ---- transform kernels (kx_fold_d.hip: double operands, kx_fold_f.hip: float)
// mode: 0 = apply_fL (rho -> phi), 1 = exchange (psi -> vxpsi);
// storage: KX_F64 / KX_F32 element type of src / psi / dst.
// The pencil pass writes one partial energy per 16-column strip into epart
// (nitems * slab/16 values) when epart is not null.
hipError_t launch_forward_d(int storage, int mode, const Geom& g, const SlabPlan& p,
                            const EigR<double>& e, const void* src, const Item* items, int nitems,
                            double* T, hipStream_t s);
// out_f: NULL = in place; else the result rounded to float into out_f (same layout)
hipError_t launch_pencil_d(const Geom& g, const PencilPlan& p, const EigR<double>& e,
                           const double* F, int nitems, double* T, double* epart, hipStream_t s,
                           float* out_f = nullptr);
// the two halves of the FP64 pencil pass around a spectral coupling step:
// dir 0: T (nitems slots) -> mode-3 coefficients S (nitems * fsize, [c][a][b]);
// dir 1: S -> T
hipError_t launch_pencil_half(int dir, const Geom& g, const EigR<double>& e, int nitems, double* T,
                              double* S, hipStream_t s);
hipError_t launch_inverse_d(int storage, int mode, const Geom& g, const SlabPlan& p,
                            const EigR<double>& e, const double* T, const Item* items, int nitems,
                            const void* psi, const double* occ, void* dst, hipStream_t s);
hipError_t launch_forward_f(int storage, int mode, const Geom& g, const SlabPlan& p,
                            const EigR<float>& e, const void* src, const Item* items, int nitems,
                            float* T, hipStream_t s);
hipError_t launch_pencil_f(const Geom& g, const PencilPlan& p, const EigR<float>& e,
                           const double* F, int nitems, float* T, double* epart, hipStream_t s);
hipError_t launch_inverse_f(int storage, int mode, const Geom& g, const SlabPlan& p,
                            const EigR<float>& e, const float* T, const Item* items, int nitems,
                            const void* psi, const double* occ, void* dst, hipStream_t s);
// ---- split-BF16 transform kernels (kx_split.hip): FP32 intermediates T
Plan make_split_plan(const Geom& g, size_t max_lds);
// Split-FP16 instead of split-BF16 (h16): the per-vector largest magnitudes
// of the forward pass's sources (omax, count of vectors) and the per-item
// largest magnitudes of the pencil's result (tmax, float bits, cleared to
// zero before the pencil launch) set the operands' power-of-two scales.
struct SplitAux {
  int h16 = 0;
  const float* omax = nullptr;
  unsigned* tmax = nullptr;
};
hipError_t launch_forward_s(int storage, int mode, const Geom& g, const SlabPlan& p,
                            const EigS& e, const void* src, const Item* items, int nitems,
                            float* T, hipStream_t s, const SplitAux& aux = SplitAux());
hipError_t launch_pencil_s(const Geom& g, const PencilPlan& p, const EigS& e, const double* F,
                           int nitems, float* T, double* epart, hipStream_t s,
                           const SplitAux& aux = SplitAux());
hipError_t launch_inverse_s(int storage, int mode, const Geom& g, const SlabPlan& p,
                            const EigS& e, const float* T, const Item* items, int nitems,
                            const void* psi, const double* occ, void* dst, hipStream_t s,
                            const SplitAux& aux = SplitAux());
// out[v] = max |x[v n .. v n + n)| for v < count (storage KX_F64 or KX_F32)
hipError_t launch_absmax(const void* x, int storage, long long n, int count, float* out,
                         hipStream_t s);
// Let kernel fn take `lds` bytes of dynamic LDS (above the 64 KiB default).
// The attribute is set once per kernel and device and remembered, so that a
// launch recorded into a graph makes no further runtime call for it.
void allow_dynamic_lds(const void* fn, size_t lds);
// zero `bytes` (a multiple of 4, 4-byte aligned) with a kernel, so that the
// clearing can be recorded into a graph
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
// flag[0] = 1 if any of the n values at x (storage KX_F64 / KX_F32) is not
// finite, else 0 (cleared by a kernel first)
hipError_t launch_nonfinite(const void* x, int storage, long long n, unsigned* flag, hipStream_t s);
// tuning helpers: index-hash values in [-1, 1); count of differing words
hipError_t launch_pattern(void* p, long long n, bool dbl, hipStream_t s);
hipError_t launch_diff(const void* a, const void* b, size_t bytes, unsigned long long* count,
                       hipStream_t s);
// b[k] = (float)a[k] and a[k] = b[k] widened, k < n (16-byte aligned arrays)
hipError_t launch_narrow(const double* a, float* b, long long n, hipStream_t s);
hipError_t launch_widen(const float* a, double* b, long long n, hipStream_t s);
// per-item energies: pair_e[index(i, j)] = dV * sum_s epart[k*nstrips + s]
hipError_t launch_pair_energy(const double* epart, int nstrips, const Item* items, int nitems,
                              int norb, double dV, double* pair_e, hipStream_t s);
// E_x = -1/4 sum_{i<=j} m_ij occ_i occ_j pair_e, m = 1 (i == j) or 2
hipError_t launch_exchange_energy(const double* pair_e, const double* occ, int norb, double* ex,
                                  hipStream_t s);

// ---- multipole boundary values (kx_multipole.hip)
constexpr int kMaxMultipoleL = 6;        // largest expansion order
constexpr int kMaxMultipoleGroups = 256;  // point groups per field of the moment reduction
// point groups of the moment reduction of an N-point field
int multipole_groups(long long N);
// dst[b] = rho[b] + c_b / (4 pi) for nb fields (storage KX_F64 / KX_F32): c_b
// from the multipole expansion (order lmax, about centre) of field b's charge,
// evaluated at the nodes outside the grid that the stencil w[0..m] reaches.
// part: nb * multipole_groups(N) * (lmax+1)^2 doubles; mom: nb * (lmax+1)^2.
hipError_t launch_multipole_rhs(int storage, const void* rho, void* dst, int nb, const Geom& g,
                                const double h[3], const double centre[3], const double* w, int m,
                                int lmax, double* part, double* mom, hipStream_t s);

// ---- Brillouin-zone sampling (kx_bloch.hip), FP64
constexpr int kMaxStencil = 12;  // largest stencil half width (order 24)
constexpr int kMaxKpoints = 64;  // largest k-point count of one exchange application
// one axis of the folded eigenbasis, for the Bloch coupling tables
struct BlochAxis {
  int n, me, mo, pe, po, periodic;
  double h;
  const double* VE;  // [i][a] pe x pe, as EigR
  const double* VO;
  const double* lamE;
  const double* lamO;
  const int* part;   // per blocked index: the coupled mode of the other parity, or -1
};
struct BlochAxes {
  BlochAxis ax[3];
  double w[kMaxStencil + 1];  // centred second-derivative weights w_0 .. w_m
  double d[kMaxStencil + 1];  // centred first-derivative weights d_1 .. d_m at d[1..m]
  int m;
  // lattice-coordinate metric g_ab of a non-orthogonal cell (nonorth = 1):
  // -L = sum_a g_aa (-L_a) - sum_{a != b} g_ab D_a D_b
  double gm[3][3];
  int nonorth;
  ZeroMode zero;  // the unscreened kernel's zero-mode value
};
// reduced phases theta_a / (2 pi) of a batch of fields, per axis
struct BlochT {
  double t[3];
};
// The items of one launch of the k-point exchange: the state pairs
// (P1, P2), P1 <= P2 < M, of one tile of kTileR rows (P1 = r0 + r) and
// kTileC columns (P2 = c0 + c), numbered in row-major order over the tile's
// valid pairs; states are P = k-point * norb + band, and a pair's class is
// k(P2) * K + k(P1).  With M == 0 the items are fields of class cls0.
constexpr int kTileR = 4, kTileC = 8;  // r0 a multiple of kTileR, c0 of kTileC
struct PairMap {
  int r0, c0;
  int M, norb, K, cls0;
};
// valid pairs of the tile at (r0, c0)
__host__ __device__ inline int tile_pairs(int r0, int c0, int M) {
  int n = 0;
  for (int r = 0; r < kTileR; ++r)
    for (int c = 0; c < kTileC; ++c) {
      const int P1 = r0 + r, P2 = c0 + c;
      n += (P1 < M && P2 < M && P1 <= P2) ? 1 : 0;
    }
  return n;
}
// the representative blocked indices per axis (unpaired modes and the even
// member of each coupled pair): one coupling group each, R[a] per axis
struct RepMap {
  const int* rep[3];
  int R[3];
};
// waves of one coupling launch (its energy partials per item)
int bloch_couple_waves(const RepMap& rm);
// Coupling tables per class (theta = 2 pi (kq[ki] - kq[qi]), cls = ki * K + qi)
// and axis, kBlochTab arrays of pmax values each at
// tab[((cls * 3 + axis) * kBlochTab + r) * pmax + idx]: r = 0 A (diagonal of
// -M), 1 b (its pair coupling, at the even member), 2 Q (the first-derivative
// circulant's imaginary diagonal), 3 R (its real pair coupling, at the even
// member); Q and R only on a non-orthogonal cell.
constexpr int kBlochTab = 4;
hipError_t launch_bloch_table(const BlochAxes& B, const double* kq, int K, int pmax, double* tab,
                              hipStream_t s);
// the spectral coupling of nitems complex items (real / imaginary spectra in
// S[2 item], S[2 item + 1], fsize each), in place; energy partials per item
hipError_t launch_bloch_couple(const BlochAxes& B, const Geom& g, const RepMap& rm,
                               const double* tab, int pmax, int kernel, double omega,
                               const PairMap& pm, int nitems, double* S, double* part,
                               hipStream_t s);
// dir 0: interleaved complex fields -> ramp-free planar pairs; dir 1: back
hipError_t launch_bloch_fields(int dir, const Geom& g, const BlochT& th, int nb, const double* in,
                               double* out, hipStream_t s);
// dir 0: psi (interleaved) -> planar u, W = 0; dir 1: W -> Vx psi (interleaved, into U)
hipError_t launch_bloch_orbitals(int dir, const Geom& g, int M, int norb, const double* kq,
                                 const double* in, double* U, double* W, hipStream_t s);
hipError_t launch_bloch_products(const Geom& g, const double* U, const PairMap& pm, int nb,
                                 double* Z, hipStream_t s);
hipError_t launch_bloch_update(const Geom& g, const double* U, const double* Z, const PairMap& pm,
                               int nb, const double* occw, double* W, hipStream_t s);
// pairE[index(P1, P2)] (row-major upper triangle of M states) of the launch's items
hipError_t launch_bloch_pair_sums(const double* part, int nblk, int nitems, const PairMap& pm,
                                  double dV, double* pairE, hipStream_t s);
hipError_t launch_bloch_energy(const double* pairE, int M, const double* occw, double* ex,
                               hipStream_t s);

// the isolated-system exchange (kx_multipole.hip): Z[b] = psi_i psi_j for
// items[b] (FP64); E_x = 1/4 dV sum_j occ_j <psi_j, vx_j> into ex, with
// part holding norb * vx_energy_parts() partial sums
hipError_t launch_pair_fields(int storage, const void* psi, const Item* items, int nb, long long N,
                              double* Z, hipStream_t s);
int vx_energy_parts();
hipError_t launch_vx_energy(int storage, const void* psi, const void* vx, int norb, long long N,
                            const double* occ, double dV, double* part, double* ex,
                            hipStream_t s);

// ---- compressed exchange algebra (kx_ace.hip); fields are rows of N values
// point-range groups for a gram of na x nb (partials <= 128 MB)
long long ace_groups(long long N, int na, int nb);
// out[i][j] = scale * sum_r A[i][r] B[j][r] (part: ngrp * na * nb doubles)
hipError_t launch_gram(int storage, const void* A, int na, const void* B, int nb, long long N,
                       long long ngrp, double* part, double scale, double* out, hipStream_t s);
// A = L L^T in place (lower), Linv = L^{-1}; status = 0 or (failed pivot + 1)
hipError_t launch_chol_inv(double* A, int n, double* Linv, int* status, hipStream_t s);
// Out[v][r] = alpha * sum_k C[v ldv + k ldk] X[k][r]
hipError_t launch_combine(int storage, const double* C, long long ldv, long long ldk, int m, int n,
                          const void* X, long long N, double alpha, void* Out, hipStream_t s);

// Pair k of round r (0 <= r < m - 1, 0 <= k < m / 2) of the round-robin
// tournament on m (even) players: player 0 stays, the others rotate.  Returns
// (min, max) of the two players; a player >= norb is the dummy of an odd
// orbital count.
__host__ __device__ inline Item rr_pair(int m, int r, int k) {
  const int pa = k, pb = m - 1 - k;
  const int p0 = (pa == 0) ? 0 : 1 + (pa - 1 + r) % (m - 1);
  const int q0 = 1 + (pb - 1 + r) % (m - 1);
  Item it;
  it.i = p0 < q0 ? p0 : q0;
  it.j = p0 < q0 ? q0 : p0;
  return it;
}

// The launch order of the symmetric pairs of norb orbitals: the norb diagonal
// pairs (i, i), then the m - 1 rounds of the tournament (m = norb rounded up to
// even), each holding floor(norb / 2) disjoint pairs.  Written on the device
// (npairs items), so that an exchange application can be recorded into a
// graph without a host transfer.
hipError_t launch_schedule(int norb, Item* out, hipStream_t s);
// out[b] = (b, -1) for b < n (the items of a batch of fields)
hipError_t launch_field_items(int n, Item* out, hipStream_t s);
// dst[k] = vals[k] for k < n, the values travelling as kernel arguments (no
// host transfer, so the copy can be recorded into a graph)
hipError_t launch_put_doubles(const double* vals, int n, double* dst, hipStream_t s);

__host__ __device__ inline long long pair_index(int i, int j, int norb) {
  // i <= j, row-major upper triangle
  return (long long)i * norb - (long long)i * (i - 1) / 2 + (j - i);
}

}  // namespace kx
