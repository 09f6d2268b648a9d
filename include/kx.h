/*
 * kx — Kronecker-product exact exchange on AMD MI355X (gfx950).
 *
 * C ABI of the HIP library libkx.so.  It applies functions of the real-space
 * finite-difference Laplacian through its Kronecker factorisation (Jing &
 * Suryanarayana, "Efficient real space formalism for hybrid density
 * functionals", Sec. III, Eqs. (11)-(21)) and uses them to apply the
 * exact-exchange operator to a set of orbitals (Sec. II, Eqs. (3)-(5) and
 * (8)-(10)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid layout: a field on an n1 x n2 x n3 grid is a contiguous array indexed
 *   idx = i1 + n1*(i2 + n2*i3)   (axis 1 fastest);
 * item b of a batch (or orbital j) starts at b*N, N = n1*n2*n3.
 * Laplacian: L = I3 (x) I2 (x) L1 + I3 (x) L2 (x) I1 + L3 (x) I2 (x) I1 (Eq. (12)),
 *   L_k the centred FD second-derivative matrix of even order fd_order on n_k
 *   nodes of spacing h_k.  Dirichlet axes are homogeneous (values outside the
 *   n_k nodes are zero); periodic axes wrap the stencil.
 * Kernels f on the spectrum lam >= 0 of -L:
 *   KX_KERNEL_COULOMB  f(lam) = 4 pi / lam                      (Eq. (5))
 *   KX_KERNEL_ERFC     f(lam) = 4 pi (1 - exp(-lam/(4 w^2))) / lam,
 *                      f(0) = pi / w^2                         (Eq. (10); the
 *                      screened Coulomb kernel erfc(w r)/r, whose Fourier
 *                      transform fixes the exponent constant)
 * Device pointers (*_dev) are owned by the caller, must be device memory
 * visible to the stream given at setup, and must not overlap each other.
 * Host pointers (*_host) are read or written before the call returns, except
 * where stated.
 * Work is enqueued on the handle's stream; calls return before it finishes
 * unless stated.  Calls on one handle must not run concurrently from several
 * host threads.
 * Errors: every argument is validated on the host before any device work is
 * enqueued; on an error the handle and all outputs are left unchanged and a
 * status other than KX_OK is returned.  Nothing aborts or throws across the
 * ABI.
 * Diagnostics (environment, read once): KX_LOG=1 prints one line per set-up,
 * tuned plan, workspace growth and application on stderr; KX_ROCTX=1 makes
 * every entry point that enqueues work a roctx range (rocprofv3
 * --marker-trace), the roctx library being looked up at run time.
 */
#ifndef KX_H
#define KX_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KX_OK = 0,
  KX_ERR_INVALID_ARG = 1,   /* bad size, spacing, order, enum, pointer or count */
  KX_ERR_UNSUPPORTED = 2,   /* valid request the library does not implement     */
  KX_ERR_SINGULAR = 3,      /* unscreened kernel with a zero eigenvalue of -L   */
  KX_ERR_OUT_OF_MEMORY = 4, /* device allocation failed, or the fixed scratch
                             * array is too small for the request              */
  KX_ERR_DEVICE = 5,        /* a HIP runtime call failed                         */
  KX_ERR_STATE = 6,         /* workspace not reserved, or energy requested
                             * before any exchange call                         */
  KX_ERR_NUMERIC = 7        /* eigen-solver did not converge / non-finite input /
                             * compressed-exchange overlap not negative definite */
} kx_status;

typedef enum { KX_BC_DIRICHLET = 0, KX_BC_PERIODIC = 1 } kx_bc;
typedef enum { KX_KERNEL_COULOMB = 0, KX_KERNEL_ERFC = 1 } kx_kernel;
/* Arithmetic of the mode products.  The spectral scaling and the energy
 * reduction are FP64 in every mode. */
typedef enum {
  KX_PREC_FP64 = 0,    /* FP64 MFMA                                          */
  KX_PREC_FP32 = 1,    /* FP32 MFMA, FP32 intermediates                      */
  KX_PREC_BF16X3 = 2,  /* three-term BF16 split of both operands, FP32 accumulate */
  KX_PREC_FP16X3 = 3,  /* three-term FP16 split of both operands, FP32
                        * accumulate; every operand scaled by a power of two
                        * into FP16's range (V by 2^12, data by its largest
                        * magnitude per item or per wave), scaled back exactly */
  KX_PREC_MIXED = 4    /* FP64 forward transform, f scaling and energies (E_x
                        * as in FP64); the potential's back-transform and the
                        * Vx psi update in split BF16 with FP32 intermediates */
} kx_prec;
/* Storage type of psi / rho / phi / vxpsi. */
typedef enum { KX_F64 = 0, KX_F32 = 1 } kx_dtype;

/* Bytes of the fixed device scratch array of kx_apply_exchange_noalloc (one
 * per device the library runs on, held until the process ends). */
#define KX_SCRATCH_BYTES (128ull << 20)

/* Opaque handle: owns the device copies of V_k and lam_k, the f table, the
 * pair schedule and the intermediate workspace. */
typedef struct kx_grid kx_grid;

/* Build L_1, L_2, L_3 (Sec. III, Eq. (12)) and diagonalise each on the device
 * in FP64: -L_k V_k = V_k diag(lam_k), lam_k ascending (Eq. (13)).
 *   n[3]      grid points per axis, 1 <= n_k <= 160
 *   h[3]      spacings, finite and > 0
 *   fd_order  even, 2..24 (stencil radius fd_order/2)
 *   bc[3]     kx_bc per axis
 *   hip_stream  hipStream_t for all work of this handle (NULL = default stream)
 *   out       receives the handle; set only on KX_OK.
 * Synchronises the stream before returning (the eigen-solver result is
 * checked on the host).  KX_ERR_NUMERIC if the Jacobi solver does not reach
 * orthogonality ~1e-13. */
kx_status kx_setup_laplacian(const int n[3], const double h[3], int fd_order,
                             const int bc[3], void* hip_stream, kx_grid** out);

/* Reserve the workspace of later kx_apply_fL and kx_apply_exchange calls
 * (the apply calls allocate nothing).  Grows the handle's buffers so that
 *   norb > 0:  kx_apply_exchange on up to norb orbitals, and
 *   norb == 0: kx_apply_fL and kx_apply_fL_multipole on batches of fields
 *              (any batch size; fields are processed in launches of at most
 *              the handle's batch size),
 * in precision prec on storage dtype; earlier reservations are kept (a call
 * never shrinks them).  Per launch slot the intermediates take 8 bytes per
 * value of the padded grid (plus 4 for KX_PREC_MIXED); an exchange reservation
 * adds the pair schedule and pair energies (16 bytes per pair), for
 * KX_PREC_FP64 on KX_F64 storage with up to 4096 orbitals the potentials of
 * one tile of pairs
 * (64 fields of N FP64 values: the exchange then runs in two stages, see
 * kx_apply_exchange), and, for
 * reduced precision on KX_F64 storage, FP32 copies of psi and Vx psi
 * (8*norb*N bytes).  Synchronises the stream when a buffer grows; a grown
 * buffer replaces the old one, so work recorded earlier into a graph must
 * not be replayed after a call that grew the workspace.
 *   norb  0 .. 65535 */
kx_status kx_reserve(kx_grid* g, int norb, int prec, int dtype);

/* phi = f(-L) rho for a batch of fields (Eqs. (20)-(21)).
 *   kernel, omega  see above; omega > 0 required for KX_KERNEL_ERFC
 *   batch          number of fields, >= 0 (0 is a no-op)
 *   dtype          storage of rho / phi: KX_F64 or KX_F32
 *   prec           arithmetic of the mode products (kx_prec).
 *   rho_dev        batch*N input values;  phi_dev  batch*N outputs (overwritten)
 * Enqueues kernels only (no allocation, host transfer or synchronisation), so
 * the call can be recorded into a caller's HIP graph.  KX_ERR_STATE if
 * kx_reserve was not called for prec and dtype.
 * KX_ERR_SINGULAR for KX_KERNEL_COULOMB when every axis is periodic, unless
 * kx_set_zero_mode gave the zero mode a value. */
kx_status kx_apply_fL(kx_grid* g, int kernel, double omega, int batch, int dtype,
                      const void* rho_dev, void* phi_dev, int prec);

/* phi = (-L_D)^{-1} (4 pi rho + c) for a batch of charge densities on a grid
 * with vacuum on every side: the unscreened problem with Dirichlet values
 * from the multipole expansion of the Coulomb kernel, enforced through the
 * right-hand side (Sec. IV, isolated systems).  For every field, the moments
 *   A_lm + i B_lm = dV sum_r rho(r) |d|^l P_l^m(cos t) e^{i m p},  d = r - centre,
 * give the potential outside the grid,
 *   phi_ext(r) = sum_{l <= lmax} sum_{m <= l} (2 - [m = 0]) (l-m)!/(l+m)!
 *                  P_l^m(cos t) (A_lm cos m p + B_lm sin m p) / |d|^(l+1),
 * and c(x) = sum over the stencil weights w_|p| / h_k^2 that reach a node
 * outside the grid of phi_ext there.  Node i of axis k sits at i h_k.
 *   rho_dev      batch*N densities (read only)
 *   phi_dev      batch*N potentials (overwritten; not aliasing rho_dev)
 *   dtype, prec  as for kx_apply_fL; the moments and c are FP64 in every mode
 *   lmax         0 .. 6
 *   centre[3]    expansion centre (host, bohr), finite
 * KX_ERR_UNSUPPORTED unless every axis is Dirichlet.  Enqueues kernels only
 * (KX_ERR_STATE if kx_reserve(g, 0, prec, dtype) was not called). */
kx_status kx_apply_fL_multipole(kx_grid* g, int batch, int dtype, const void* rho_dev,
                                void* phi_dev, int prec, int lmax, const double centre[3]);

/* The unscreened exact exchange of an isolated system: kx_apply_exchange
 * with KX_KERNEL_COULOMB on an all-Dirichlet grid, every pair solve taking
 * its boundary values from the multipole expansion of its pair density
 * rho_ij = psi_i psi_j (the problem of kx_apply_fL_multipole: phi_ij =
 * f(-L_D)(rho_ij + c_ij / (4 pi)), Sec. IV).  The boundary values make the
 * pair solve non-symmetric, so E_x is taken from the operator,
 *   E_x = 1/4 sum_j occ_j <psi_j, (Vx psi)_j>_h,
 * which equals -1/4 sum_{i,j} occ_i occ_j (rho_ij, phi_ij)_h; read it with
 * kx_exchange_energy (kx_pair_energies then holds no pairs).
 *   norb, dtype, psi_dev, occ_host, vxpsi_dev  as for kx_apply_exchange
 *   prec         KX_PREC_FP64 (others: KX_ERR_UNSUPPORTED)
 *   lmax, centre as for kx_apply_fL_multipole
 * KX_ERR_UNSUPPORTED unless every axis is Dirichlet.  Enqueues kernels only
 * (KX_ERR_STATE without kx_reserve(g, norb, KX_PREC_FP64, dtype)). */
kx_status kx_apply_exchange_multipole(kx_grid* g, int norb, int dtype, const void* psi_dev,
                                      const double* occ_host, void* vxpsi_dev, int prec, int lmax,
                                      const double centre[3]);

/* Exact-exchange operator on norb real orbitals (Sec. II, Eqs. (3), (8)):
 *   (Vx psi)_j = - sum_i occ_i phi_ij psi_i,   phi_ij = f(-L)(psi_i psi_j),
 * evaluated over the norb(norb+1)/2 symmetric pairs i <= j; each pair
 * updates orbital j and, if i != j, orbital i.  occ_host[norb] are the
 * spin-summed occupations used as literal weights (a closed shell with
 * occ = 2 gives twice the per-spin operator of Eq. (3)).
 *   dtype, prec  as for kx_apply_fL.  With KX_PREC_FP32, KX_PREC_BF16X3,
 *              KX_PREC_FP16X3 or KX_PREC_MIXED on KX_F64 storage the orbitals are rounded to
 *              FP32 once for the inverse pass and Vx psi is accumulated in
 *              FP32 before it is widened into vxpsi_dev (the FP32 copies
 *              reserved by kx_reserve).  KX_PREC_MIXED forms the pair
 *              products and all energies from the FP64 orbitals in FP64.
 *   psi_dev    norb*N orbitals (read only)
 *   vxpsi_dev  norb*N outputs, overwritten (not accumulated into)
 * Also prepares E_x = -1/4 sum_{i,j} occ_i occ_j (rho_ij, phi_ij)_h with
 * (u,v)_h = h1 h2 h3 sum_r u v (Eqs. (4), (9)) and the per-pair energies,
 * read back by kx_exchange_energy / kx_pair_energies.  The reduction order is
 * fixed: results are bitwise reproducible run to run, and do not depend on
 * the batch size.
 * Enqueues kernels only: the f table, the pair schedule and the occupations
 * (as kernel arguments) are written by kernels, so the call allocates
 * nothing, makes no host transfer or synchronisation and can be recorded
 * into a caller's HIP graph (the recorded work carries occ_host's values).
 * KX_ERR_STATE if kx_reserve was not called for at least norb orbitals in
 * prec and dtype.
 * With KX_PREC_FP64 on KX_F64 storage (up to 4096 orbitals) the pairs run in
 * tiles of 8 x 8 orbitals in two stages: the transforms write the tile's
 * potentials, and one kernel applies them to Vx psi, reading and writing
 * each orbital of the tile once (the other cases update Vx psi in the
 * inverse pass, two orbitals per pair).  Either way results do not depend
 * on the batch size. */
kx_status kx_apply_exchange(kx_grid* g, int kernel, double omega, int norb, int dtype,
                            const void* psi_dev, const double* occ_host, void* vxpsi_dev,
                            int prec);

/* kx_apply_exchange for callers that cannot allocate device memory (code
 * under HIP graph capture that must not grow the handle, tight serving
 * loops, harnesses that forbid allocation): the same arguments, results and
 * arithmetic, with every per-call buffer (intermediates, energy partials,
 * pair schedule, pair energies, occupations, FP16 scales) carved out of a
 * fixed device array of KX_SCRATCH_BYTES per device instead of the handle's
 * workspace; kx_reserve is not needed.  No FP32 working copies: reduced
 * precisions on KX_F64 storage read and update the caller's FP64 arrays
 * directly, and Vx psi accumulates in FP64.  The FP64 path keeps the fused
 * inverse pass (no room for a tile's potentials), so its Vx psi equals
 * kx_apply_exchange's to rounding (the pair energies and E_x bitwise).
 * Launches take as many pairs as fit in the array (up to the handle's batch
 * size).
 * KX_ERR_OUT_OF_MEMORY if the schedule, pair energies and one launch slot
 * (at 96^3 about 7 MB in FP64) do not fit in KX_SCRATCH_BYTES.
 * Every call on one device shares that device's array and leaves its
 * contents there: calls that overlap on one device (other streams, other
 * host threads) race and must not be issued; kx_pair_energies reads the
 * array, so it reports the last call only until another call on the device. */
kx_status kx_apply_exchange_noalloc(kx_grid* g, int kernel, double omega, int norb, int dtype,
                                    const void* psi_dev, const double* occ_host,
                                    void* vxpsi_dev, int prec);

/* ---- Brillouin-zone sampling (Sec. II: the pair (m q, n k) satisfies Bloch
 * boundary conditions at the wavevector k - q on the periodic axes).
 * A periodic axis of n nodes with the phase theta wraps its stencil as
 * u(x + n h) = e^{i theta} u(x); -L(theta) is Hermitian and f(-L(theta)) is
 * applied in the real eigenbasis of the theta = 0 grid, where it couples the
 * even and odd mode of each frequency (2 x 2 blocks per axis).  Complex
 * fields are interleaved (re, im) doubles, layout [field][n3][n2][n1].
 * Only KX_PREC_FP64 is implemented (other precisions: KX_ERR_UNSUPPORTED).
 * Node i of an axis sits at i h. */

/* Non-orthogonal cells (Sec. III, closing remark): lattice[9] holds, row a,
 * the direction of lattice axis a (any length; node i of axis a sits at
 * i h_a along it).  With E the unit directions as columns, the Laplacian in
 * lattice coordinates is
 *   sum_ab g_ab d^2/(dxi_a dxi_b),  g = E^-1 E^-T,
 * discretised as sum_a g_aa L_a + sum_{a != b} g_ab D_a D_b with D_a the
 * centred first-derivative matrix of the same order (weights
 * d_p = (-1)^(p+1) (m!)^2 / (p (m-p)! (m+p)!)), and the volume element is
 * h1 h2 h3 |det E|.  Requires periodic conditions on every axis
 * (KX_ERR_UNSUPPORTED otherwise: D_a and L_a do not commute with Dirichlet
 * ends).  A non-orthogonal cell is served by the Bloch entry points below
 * (use the Gamma point, theta = 0, for real orbitals) and kx_ace_build /
 * kx_ace_apply; kx_apply_fL and the real exchange calls return
 * KX_ERR_UNSUPPORTED while it is set.  lattice == NULL (or orthonormal
 * directions) restores the orthogonal cell.  KX_ERR_INVALID_ARG for
 * non-finite, zero or (nearly) coplanar directions (|det E| <= 1e-6).
 * Work recorded into a graph before the call must not be replayed after it. */
kx_status kx_set_cell(kx_grid* g, const double lattice[9]);

/* The value of the unscreened kernel at the zero mode (Sec. IV: for 3D bulk
 * systems the k = q problem is singular, and the paper takes the value from
 * auxiliary functions; the library applies a value the caller computes).
 * With enable = 1, KX_KERNEL_COULOMB on a grid whose spectrum contains 0
 * (every axis periodic; for the Bloch calls, phases that are multiples of
 * 2 pi) is solved with f = value on the zero mode (the constant, or its
 * ramp) instead of returning KX_ERR_SINGULAR: phi = (-L)^+ 4 pi rho + value
 * mean(rho).  The zero mode is recognised as an eigenvalue sum below 1e-9
 * of the largest.  enable = 0 restores KX_ERR_SINGULAR.  Applies to every
 * entry point and precision (the f table is FP64).  Work recorded into a
 * graph before the call must not be replayed after it. */
kx_status kx_set_zero_mode(kx_grid* g, int enable, double value);

/* Opt-in checks.  KX_CHECK_FINITE: kx_apply_fL, kx_apply_fL_multipole,
 * kx_apply_exchange, kx_apply_exchange_noalloc, kx_apply_fL_bloch and
 * kx_apply_exchange_bloch scan their input fields before enqueueing any work
 * and return KX_ERR_NUMERIC (nothing written) if a value is NaN or infinite;
 * after the work they scan the outputs (and E_x) and return KX_ERR_NUMERIC
 * if one is (the outputs then hold the computed values).  With the check on
 * these calls synchronise the stream and cannot be recorded into a graph
 * (KX_ERR_STATE while the stream is capturing).  flags: 0 or KX_CHECK_FINITE. */
#define KX_CHECK_FINITE 1
kx_status kx_set_checks(kx_grid* g, int flags);

/* Reserve the buffers of the Bloch calls below: nk == 0 for
 * kx_apply_fL_bloch alone, else for kx_apply_exchange_bloch on nk k-points of
 * norb bands (and kx_apply_fL_bloch).  Builds, once per handle, the map of
 * coupled modes from the eigenvectors (synchronises; KX_ERR_NUMERIC if the
 * eigenbasis does not split into such pairs).  Grows buffers as kx_reserve
 * does: a launch's fields and spectra (16 bytes per padded-grid value per
 * item, 32 items), and for the exchange 32 bytes per grid point per state
 * (ramp-free copies of psi and Vx psi) plus 8 per state pair.
 *   nk  0 .. 64;  nk * norb <= 65535 */
kx_status kx_reserve_bloch(kx_grid* g, int nk, int norb);

/* phi = f(-L(theta)) rho for a batch of complex fields with the Bloch
 * phases theta[3] (host, radians, one per axis; 0 on Dirichlet axes, else
 * KX_ERR_INVALID_ARG).  rho_dev, phi_dev: batch interleaved complex fields
 * (not aliasing).  KX_ERR_SINGULAR for KX_KERNEL_COULOMB when every axis is
 * periodic with theta a multiple of 2 pi.  Enqueues kernels only
 * (KX_ERR_STATE without kx_reserve_bloch). */
kx_status kx_apply_fL_bloch(kx_grid* g, int kernel, double omega, int batch, const double theta[3],
                            const void* rho_dev, void* phi_dev, int prec);

/* Exact exchange with k-point sampling for one spin channel (Sec. II):
 *   (Vx psi)_nk = - sum_{m q} w_q occ_mq psi_mq phi_{mq,nk},
 *   -L(2 pi (k - q)) phi_{mq,nk} = 4 pi conj(psi_mq) psi_nk   (f for erfc),
 *   E_x = -1/4 sum_{nk, mq} w_k w_q occ_nk occ_mq (rho_{mq,nk}, phi_{mq,nk})_h,
 * solved once per unordered pair of states (phi_{nk,mq} = conj(phi_{mq,nk})).
 *   nk               1 .. 64 k-points; kpts_host[nk][3] reduced coordinates
 *                    (0 on Dirichlet axes); wk_host[nk] weights
 *   norb             bands per k-point; occ_host[nk][norb] occupations
 *   psi_dev          [nk][norb] interleaved complex fields psi_nk(x)
 *   vxpsi_dev        the same layout, overwritten with (Vx psi)_nk
 * Spin: one call per channel with that channel's occupations.  E_x is read
 * with kx_exchange_energy (kx_pair_energies then holds no pairs).  Results
 * do not depend on the handle's batch size.  Enqueues kernels only
 * (KX_ERR_STATE without kx_reserve_bloch for at least nk * norb states). */
kx_status kx_apply_exchange_bloch(kx_grid* g, int kernel, double omega, int nk, int norb,
                                  const double* kpts_host, const double* wk_host,
                                  const double* occ_host, const void* psi_dev, void* vxpsi_dev,
                                  int prec);

/* Ragged batch: the exact-exchange application of nsys independent systems
 * (each its own handle, grid, boundary conditions, kernel, omega, orbital
 * count), recorded once into one HIP graph with one branch per system and
 * replayed by a single graph launch while the handles, their buffers and
 * the arguments below are unchanged (recorded again otherwise).
 *   grids[nsys]      distinct handles (each owns its workspace)
 *   kernels, omegas, norbs   per system, as for kx_apply_exchange
 *   dtype, prec      shared by all systems
 *   psi_dev, occ_host, vxpsi_dev  per system, as for kx_apply_exchange
 *   ex_out           NULL or nsys doubles: E_x per system
 * Reserves each handle's workspace as kx_reserve does.
 * Synchronises before returning; afterwards kx_exchange_energy and
 * kx_pair_energies on each handle report that system.  Validation and all
 * allocation happen before any recorded work; on error no system is
 * partially updated except through a device failure (KX_ERR_DEVICE).
 * The recorded graph lives with grids[0] and is released by kx_destroy. */
kx_status kx_batch_apply_exchange(int nsys, kx_grid* const* grids, const int* kernels,
                                  const double* omegas, const int* norbs, int dtype,
                                  const void* const* psi_dev, const double* const* occ_host,
                                  void* const* vxpsi_dev, int prec, double* ex_out);

/* Autotuner: time every launch shape the transform kernels accept for this
 * grid (workgroup z-slabs, staging chunk rows, V blocks in LDS or not,
 * parity split, pencil waves) for precision prec on storage dtype (the
 * split precisions share one set of shapes, tuned with BF16X3), on
 * synthetic data in batches of `items` pairs (<= 0: the handle's batch size),
 * and keep the fastest per pass for later calls on this handle.
 *   verify      non-zero: also check that every shape gives bitwise the same
 *               intermediate and Vx psi as the current one (KX_ERR_NUMERIC
 *               otherwise; the plan is then left unchanged); no cache use
 *   cache_path  NULL, or a text file: a line for this grid shape, precision
 *               and device is read instead of timing (accepted only if the
 *               shape is one the planner proposes); a new result is appended
 * Allocates temporary device buffers (2*items orbitals in and out) and
 * synchronises the stream. */
kx_status kx_autotune(kx_grid* g, int prec, int dtype, int items, int verify,
                      const char* cache_path);

/* The launch shapes in use for prec (a test and reporting hook):
 * fwd_out[6] = {parity split, z-slabs, waves, chunk rows, V in LDS, LDS bytes},
 * pen_out[3] = {waves, LDS bytes, items per wave of the pipelined pencil
 * (0: one item per wave)}, inv_out[6] like fwd_out (parity split 1). */
kx_status kx_get_plan(kx_grid* g, int prec, int* fwd_out, int* pen_out, int* inv_out);

/* E_x of the last kx_apply_exchange on this handle.  Synchronises the stream.
 * KX_ERR_STATE if there was none. */
kx_status kx_exchange_energy(kx_grid* g, double* ex_out);

/* e_ij = (rho_ij, phi_ij)_h of the last kx_apply_exchange for npairs pairs
 * given as pairs_host[2k] = i, pairs_host[2k+1] = j (any order of i, j).
 * Synchronises the stream.  A test hook for sampled-pair checks. */
kx_status kx_pair_energies(kx_grid* g, int npairs, const int* pairs_host, double* e_out_host);

/* Exact exchange in adaptively compressed (ACE) form (Sec. IV: the exchange
 * operator enters the self-consistent iteration through the compressed
 * operator of Lin, J. Chem. Theory Comput. 12, 2242 (2016)).  From the
 * orbitals psi and W = Vx psi (the output of kx_apply_exchange):
 *   M = (psi_j, W_k)_h  (norb x norb),  -M = L L^T  (Cholesky, L lower with a
 *   positive diagonal),  xi = L^{-1} W,
 * so that V_ACE phi = -sum_k xi_k (xi_k, phi)_h equals Vx on the span of the
 * orbitals.  FP64 arithmetic; fields stored as dtype (KX_F64 / KX_F32).
 *   norb        1 .. min(1024, N)
 *   psi_dev, w_dev  norb*N device fields, orbital k at k*N
 *   xi_dev      norb*N device output (not aliasing psi_dev or w_dev)
 * KX_ERR_NUMERIC if -M is not positive definite (xi is not written then).
 * Synchronises the stream once (to read the factorisation status).  The
 * small matrices and partial sums live in the handle, grown here to also
 * cover kx_ace_apply on up to 4096 fields with up to norb vectors. */
kx_status kx_ace_build(kx_grid* g, int norb, int dtype, const void* psi_dev, const void* w_dev,
                       void* xi_dev);

/* out_v = V_ACE phi_v = -sum_k xi_k (xi_k, phi_v)_h for nvec fields.
 *   xi_dev      norb*N (from kx_ace_build), phi_dev nvec*N, out_dev nvec*N
 *               (out_dev must not alias xi_dev or phi_dev); nvec 1 .. 4096
 * Enqueued on the handle's stream: no allocation or synchronisation.
 * KX_ERR_STATE if no kx_ace_build on this handle had at least norb orbitals. */
kx_status kx_ace_apply(kx_grid* g, int norb, int dtype, const void* xi_dev, int nvec,
                       const void* phi_dev, void* out_dev);

/* The compressed exchange of one k-point (Sec. IV with the k-point exchange
 * of Sec. II): complex Bloch orbitals psi_nk and W = (Vx psi)_nk of that k
 * (from kx_apply_exchange_bloch), norb interleaved complex fields each.
 *   M = (psi_j, W_k)_h (Hermitian, negative definite), -M = L L^H,
 *   xi = W L^{-H},  V_ACE phi = -sum_k xi_k (xi_k, phi)_h.
 * The algebra runs on the real form: a complex field of N values is a real
 * vector of 2 N, the span of the orbitals is spanned by the 2 norb real
 * vectors {psi_j, i psi_j}, and the real compressed operator built on them
 * (kx_ace_build's kernels) is the complex one.  xi_dev receives those
 * 2 norb real vectors, i.e. 2 norb complex fields (pass them to
 * kx_ace_apply_complex with the same norb).  FP64; 1 <= norb <= 512.
 * Grows its buffers (the real forms, 64 bytes per grid point and orbital)
 * and synchronises once, as kx_ace_build. */
kx_status kx_ace_build_complex(kx_grid* g, int norb, const void* psi_dev, const void* w_dev,
                               void* xi_dev);

/* out_v = V_ACE phi_v for nvec interleaved complex fields (1 .. 4096), with
 * xi_dev from kx_ace_build_complex (2 norb complex fields).  Enqueued only;
 * KX_ERR_STATE if no build covered norb. */
kx_status kx_ace_apply_complex(kx_grid* g, int norb, const void* xi_dev, int nvec,
                               const void* phi_dev, void* out_dev);

/* Copy lam_axis (n_axis values, ascending) and V_axis (n_axis x n_axis,
 * row-major, V[i*n + a] = component i of eigenvector a) to the host.  Either
 * output may be NULL.  Synchronises the stream.  A test hook. */
kx_status kx_get_eigensystem(kx_grid* g, int axis, double* lam_host, double* V_host);

/* Optional launch timing.  kx_profile(g, 1) clears the record and brackets
 * every later kernel launch of this handle with hipEvents on its stream;
 * kx_profile(g, 0) stops.  kx_profile_read returns the summed elapsed time and
 * the launch count of one phase since the last kx_profile(g, 1).  Both
 * synchronise the stream. */
typedef enum {
  KX_PHASE_FORWARD = 0,  /* pair product + modes 2, 1 (per z-slab)          */
  KX_PHASE_PENCIL = 1,   /* mode 3, f(Lambda) scaling + energy, mode 3 back  */
  KX_PHASE_INVERSE = 2,  /* modes 1, 2 back + Vx psi accumulation            */
  KX_PHASE_ENERGY = 3,   /* deterministic energy reductions                  */
  KX_PHASE_ACCUM = 4     /* Vx psi from the stored potentials (FP64 exchange) */
} kx_phase;
kx_status kx_profile(kx_grid* g, int enable);
kx_status kx_profile_read(kx_grid* g, int phase, double* total_ms, long long* launches);
/* As kx_profile(g, 1), but brackets only the launches of the phases whose bit
 * (1 << KX_PHASE_*) is set in mask (1..31).  Each pair of events makes the
 * stream drain between the launches it separates, so timing one phase
 * disturbs a run less than timing all of them. */
kx_status kx_profile_phases(kx_grid* g, int mask);

/* Free every device allocation of the handle (after synchronising its stream).
 * NULL is accepted. */
kx_status kx_destroy(kx_grid* g);

/* Static English text for a status code. */
const char* kx_status_string(int status);

/* ---- host-only helpers: no device is touched; usable without a GPU ---- */

/* Centred FD weights for d^2/dx^2 of order fd_order (Sec. III): w_out[0..m],
 * m = fd_order/2, with h^2 f''(x) ~ w0 f(x) + sum_p w_p (f(x+ph) + f(x-ph)). */
kx_status kx_fd_weights(int fd_order, double* w_out);

/* The 1-D matrix L_k (n x n, row-major, includes the 1/h^2) of Eq. (12). */
kx_status kx_laplacian_1d(int n, double h, int fd_order, int bc, double* L_out);

/* The pair schedule used by kx_apply_exchange: the symmetric pairs grouped
 * into batches in which no orbital appears in two different pairs, so every
 * batch can update vxpsi without atomics.  With pairs_out == NULL only the
 * counts are returned.  pairs_out receives 2*npairs ints (i, j),
 * batch_offsets_out nbatches+1 offsets into it; max_batch caps the batch size
 * (<= 0: no cap). */
kx_status kx_pair_schedule(int norb, int max_batch, int* npairs_out, int* nbatches_out,
                           int* pairs_out, int* batch_offsets_out);

#ifdef __cplusplus
}
#endif
#endif /* KX_H */
