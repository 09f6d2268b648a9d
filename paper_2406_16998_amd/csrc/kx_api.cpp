// Host side of the kx C ABI: argument validation, FD weights and 1-D
// Laplacian assembly (Sec. III, Eq. (12)), the pair schedule, workspace
// management and the launch sequence of the transform kernels.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "kx_aux.h"
#include "kx_internal.h"

using namespace kx;

// ============================================================ host helpers
namespace {

bool valid_order(int order) { return order >= 2 && order <= 24 && order % 2 == 0; }

// ---- diagnostics
// KX_LOG=1: one line per set-up, plan, workspace growth and application on
// stderr.  KX_ROCTX=1: every entry point that enqueues work is a roctx range
// (visible with rocprofv3 --marker-trace); the roctx library is looked up at
// run time, so nothing is linked when the ranges are off.
bool env_on(const char* name) {
  const char* v = std::getenv(name);
  return v && v[0] && !(v[0] == '0' && v[1] == 0);
}
bool log_on() {
  static const bool on = env_on("KX_LOG");
  return on;
}
void kx_logf(const char* fmt, ...) {
  if (!log_on()) return;
  va_list ap;
  va_start(ap, fmt);
  std::fputs("[kx] ", stderr);
  std::vfprintf(stderr, fmt, ap);
  std::fputc('\n', stderr);
  va_end(ap);
}
struct Roctx {
  int (*push)(const char*) = nullptr;
  int (*pop)() = nullptr;
  Roctx() {
    if (!env_on("KX_ROCTX")) return;
    void* h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
    if (!h) h = dlopen("libroctx64.so.4", RTLD_NOW | RTLD_LOCAL);
    if (!h) return;
    push = reinterpret_cast<int (*)(const char*)>(dlsym(h, "roctxRangePushA"));
    pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
    if (!push || !pop) push = nullptr, pop = nullptr;
  }
};
const Roctx& roctx() {
  static const Roctx r;
  return r;
}
struct Range {
  const bool on;
  explicit Range(const char* name) : on(roctx().push != nullptr) {
    if (on) roctx().push(name);
  }
  ~Range() {
    if (on) roctx().pop();
  }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};
const char* prec_name(int prec) {
  static const char* names[] = {"fp64", "fp32", "bf16x3", "fp16x3", "mixed"};
  return prec >= 0 && prec <= 4 ? names[prec] : "?";
}

// Closed form of the centred second-derivative weights of order 2m:
//   w_p = 2 (-1)^(p+1) (m!)^2 / (p^2 (m-p)! (m+p)!),   w_0 = -2 sum_{p>=1} w_p.
// The factorial ratio is accumulated as a product to stay in range.
void fd_weights_closed_form(int order, double* w) {
  const int m = order / 2;
  double s = 0.0;
  for (int p = 1; p <= m; ++p) {
    // (m!)^2 / ((m-p)! (m+p)!) = prod_{k=1..p} (m-p+k) / (m+k)
    double ratio = 1.0;
    for (int k = 1; k <= p; ++k) ratio *= double(m - p + k) / double(m + k);
    const double sign = (p % 2 == 1) ? 1.0 : -1.0;
    w[p] = 2.0 * sign * ratio / (double(p) * double(p));
    s += w[p];
  }
  w[0] = -2.0 * s;
}

// Closed form of the centred first-derivative weights of order 2m:
//   d_p = (-1)^(p+1) (m!)^2 / (p (m-p)! (m+p)!),  d_{-p} = -d_p,  p = 1..m,
// into d[1..m] (d[0] = 0); the factorial ratio accumulated as a product.
void fd_weights_d1_closed_form(int order, double* d) {
  const int m = order / 2;
  d[0] = 0.0;
  for (int p = 1; p <= m; ++p) {
    double r = 1.0;
    for (int j = 1; j <= p; ++j) r *= (double)(m - j + 1) / (double)(m + j);
    d[p] = ((p % 2) ? 1.0 : -1.0) * r / p;
  }
}

void laplacian_1d(int n, double h, int order, int bc, double* L) {
  double w[13];
  fd_weights_closed_form(order, w);
  const int m = order / 2;
  const double ih2 = 1.0 / (h * h);
  std::fill(L, L + (size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    for (int p = -m; p <= m; ++p) {
      int j = i + p;
      const double v = w[p < 0 ? -p : p] * ih2;
      if (bc == KX_BC_DIRICHLET) {
        if (j >= 0 && j < n) L[(size_t)i * n + j] += v;
      } else {
        j %= n;
        if (j < 0) j += n;
        L[(size_t)i * n + j] += v;
      }
    }
  }
}

// Batch offsets of the pair schedule of norb orbitals (the launch order that
// launch_schedule writes on the device: the diagonal pairs, then the rounds of
// the round-robin tournament): each group is cut into ceil(size / cap) batches
// of near-equal size (cap <= 0: no cut).  No orbital appears twice in a batch.
void schedule_offsets(int norb, int cap, std::vector<int>& offsets) {
  offsets.clear();
  int pos = 0;
  auto cut = [&](int size) {
    if (size <= 0) return;
    const int parts = cap > 0 ? (size + cap - 1) / cap : 1;
    const int base = size / parts, extra = size % parts;
    for (int k = 0; k < parts; ++k) {
      offsets.push_back(pos);
      pos += base + (k < extra ? 1 : 0);
    }
  };
  cut(norb);
  const int m = (norb + 1) & ~1;
  for (int r = 0; r + 1 < m; ++r) cut(norb / 2);
  offsets.push_back(pos);
}

// The same order on the host (kx_pair_schedule).
void schedule_pairs(int norb, std::vector<Item>& pairs) {
  pairs.clear();
  for (int i = 0; i < norb; ++i) pairs.push_back({i, i});
  const int m = (norb + 1) & ~1;
  for (int r = 0; r + 1 < m; ++r)
    for (int k = 0; k < m / 2; ++k) {
      const Item p = rr_pair(m, r, k);
      if (p.j < norb) pairs.push_back(p);
    }
}

// Device buffers one exchange application (or one batch of fields) works in,
// with the number of values each holds.  The handle owns one set (grown only
// by kx_reserve, kx_autotune and the batch entry point); the no-allocation
// entry point carves a set out of the fixed scratch array.
struct Work {
  void* T = nullptr;         // intermediates: slots fields of Geom::slot values
  float* T2 = nullptr;       // the mixed path's FP32 copy of the pencil's result
  double* epart = nullptr;   // per-strip energy partials, slots * nstrips
  unsigned* tmax = nullptr;  // split-FP16 per-item result maxima, slots
  Item* fitems = nullptr;    // (b, -1), b < slots: the items of a batch of fields
  double* mpart = nullptr;   // multipole moment partials (all-Dirichlet grids), per slot
  double* mmom = nullptr;    // multipole moments, per slot
  double* fields = nullptr;  // pair densities of the isolated-system exchange, slots * N
  double* dpart = nullptr;   // its energy partials, norb * vx_energy_parts()
  long long dpart_cap = 0;
  int slots = 0;             // items per launch
  size_t tbytes = 0;         // bytes per slot of T (8- or 4-byte values)
  Item* items = nullptr;     // pair schedule
  long long items_cap = 0;
  double* pairE = nullptr;   // pair energies, upper-triangle index
  long long pairE_cap = 0;
  double* occ = nullptr;     // occupations
  int occ_cap = 0;
  float* omax = nullptr;     // split-FP16 per-vector largest magnitudes
  int omax_cap = 0;
  float* psi32 = nullptr;    // FP32 working copies of psi and Vx psi
  float* vx32 = nullptr;
  size_t work32_cap = 0;
  double* phi = nullptr;     // the FP64 exchange's potentials of one tile of pairs
  long long phi_cap = 0;     // (fields of N values)
};

}  // namespace

// ============================================================ the handle
struct kx_grid {
  int n[3];
  double h[3];
  int order;
  int bc[3];
  int device = 0;  // the device current at set-up
  hipStream_t stream;
  Geom geom;
  Plan plan_d, plan_f, plan_s;  // launch shapes: double / float / split-bf16 operands
  // folded eigen-blocks per axis (device): even / odd halves and transposes
  double* dVE[3] = {nullptr, nullptr, nullptr};
  double* dVO[3] = {nullptr, nullptr, nullptr};
  double* dVET[3] = {nullptr, nullptr, nullptr};
  double* dVOT[3] = {nullptr, nullptr, nullptr};
  double* dLamE[3] = {nullptr, nullptr, nullptr};
  double* dLamO[3] = {nullptr, nullptr, nullptr};
  // the same blocks rounded to float, for FP32 mode products
  float* fVE[3] = {nullptr, nullptr, nullptr};
  float* fVO[3] = {nullptr, nullptr, nullptr};
  float* fVET[3] = {nullptr, nullptr, nullptr};
  float* fVOT[3] = {nullptr, nullptr, nullptr};
  // the same blocks as three-term bf16 splits, for the split-BF16 products
  short* sVE[3] = {nullptr, nullptr, nullptr};
  short* sVO[3] = {nullptr, nullptr, nullptr};
  short* sVET[3] = {nullptr, nullptr, nullptr};
  short* sVOT[3] = {nullptr, nullptr, nullptr};
  // three-term FP16 splits of 2^12 V (split-FP16 path)
  short* hVE[3] = {nullptr, nullptr, nullptr};
  short* hVO[3] = {nullptr, nullptr, nullptr};
  short* hVET[3] = {nullptr, nullptr, nullptr};
  short* hVOT[3] = {nullptr, nullptr, nullptr};
  // full eigensystem per axis (host), lam ascending, V[i*n + a]
  std::vector<double> lam_host[3];
  std::vector<double> V_host[3];
  // f table, filled for the requested kernel by every application
  double* dF = nullptr;
  // the cell: lattice-coordinate metric and |det E| of a non-orthogonal
  // all-periodic cell (kx_set_cell); identity and 1 otherwise
  bool nonorth = false;
  // the value of the unscreened kernel at the zero mode (kx_set_zero_mode)
  ZeroMode zero;
  // opt-in checks (kx_set_checks) and their device flag
  int checks = 0;
  unsigned* dFlag = nullptr;
  double cell_g[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  double cell_jac = 1.0;
  // workspace (grown by kx_reserve) and results
  Work ws;
  // Brillouin-zone sampling: the coupled mode of every folded eigenvector
  // (built once) and the buffers of the Bloch entry points (grown by
  // kx_reserve_bloch); capacities in elements
  struct Bloch {
    int* part = nullptr;  // 3 * pmax
    int* reps = nullptr;  // 3 * pmax: representative indices per axis
    int nrep[3] = {0, 0, 0};
    int pmax = 0;
    bool mapped = false;
    double* Z = nullptr;  // fields / spectra of a launch
    long long z_cap = 0;
    double* epart = nullptr;  // coupling-kernel energy partials
    long long epart_cap = 0;
    double* tab = nullptr;  // coupling tables per class
    long long tab_cap = 0;
    double* kq = nullptr;  // reduced k-points (or phases / 2 pi)
    long long kq_cap = 0;
    double* occw = nullptr;  // w_k occ_nk per state
    long long occw_cap = 0;
    double* U = nullptr;  // ramp-free orbitals, planar
    long long u_cap = 0;
    double* W = nullptr;  // ramp-free Vx psi accumulators, planar
    long long w_cap = 0;
    double* pairE = nullptr;
    long long pairE_cap = 0;
  } bl;
  int max_slots = 64;   // largest batch of pairs / fields per launch
  int batch_cap = 64;   // pairs per launch of the exchange schedule (<= max_slots)
  double* dEx = nullptr;
  const double* last_pairE = nullptr;  // where the last application left its pair energies
  // compressed exchange: gram partial sums, the small matrix (overwritten by
  // its Cholesky factor), the factor's inverse, the (xi, phi) coefficients
  double* dAcePart = nullptr;
  long long ace_part_cap = 0;
  double* dAceA = nullptr;
  double* dAceLinv = nullptr;
  long long ace_mat_cap = 0;
  double* dAceG = nullptr;
  long long ace_g_cap = 0;
  // real forms of complex orbitals and W for the compressed exchange of k-points
  double* dAceU = nullptr;
  long long ace_u_cap = 0;
  double* dAceW = nullptr;
  long long ace_w_cap = 0;
  int ace_norb = 0;  // largest orbital count kx_ace_apply is reserved for
  int* dAceStatus = nullptr;
  int last_norb = -1;
  // optional per-launch timing (hipEvents on the handle's stream)
  bool prof_on = false;
  int prof_mask = 0x1F;  // phases whose launches are bracketed (1 << KX_PHASE_*)
  bool capturing = false;  // no timing events (the batch graph, the no-allocation path)
  bool recording = false;  // a caller records this call into a graph: timing events are
                           // recorded as graph nodes, but none is created
  // identity and buffer generation: a recorded graph bakes in device
  // addresses, so any reallocation invalidates it
  unsigned long long id = 0;
  unsigned long long gen = 0;
  // the recorded multi-system exchange whose origin stream is this handle's
  struct BatchGraph {
    std::vector<unsigned long long> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t origin = nullptr;        // capture and replay stream
    std::vector<hipStream_t> branch;     // one per system
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
  } batch;
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_kind;
};

namespace {

#define KX_HIP(call)                   \
  do {                                 \
    if ((call) != hipSuccess) {        \
      (void)hipGetLastError();         \
      return KX_ERR_DEVICE;            \
    }                                  \
  } while (0)

kx_status dev_alloc(void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return KX_ERR_OUT_OF_MEMORY;
  }
  return KX_OK;
}

void dev_free(void* p) {
  if (p) (void)hipFree(p);
}

EigR<double> eig_of(const kx_grid* g) {
  EigR<double> e;
  for (int k = 0; k < 3; ++k) {
    e.VE[k] = g->dVE[k];
    e.VO[k] = g->dVO[k];
    e.VET[k] = g->dVET[k];
    e.VOT[k] = g->dVOT[k];
  }
  return e;
}

EigR<float> eigf_of(const kx_grid* g) {
  EigR<float> e;
  for (int k = 0; k < 3; ++k) {
    e.VE[k] = g->fVE[k];
    e.VO[k] = g->fVO[k];
    e.VET[k] = g->fVET[k];
    e.VOT[k] = g->fVOT[k];
  }
  return e;
}

EigS eigs_of(const kx_grid* g) {
  EigS e;
  for (int k = 0; k < 3; ++k) {
    e.E[k] = g->sVE[k];
    e.O[k] = g->sVO[k];
    e.ET[k] = g->sVET[k];
    e.OT[k] = g->sVOT[k];
  }
  return e;
}

EigS eigh_of(const kx_grid* g) {
  EigS e;
  for (int k = 0; k < 3; ++k) {
    e.E[k] = g->hVE[k];
    e.O[k] = g->hVO[k];
    e.ET[k] = g->hVET[k];
    e.OT[k] = g->hVOT[k];
  }
  return e;
}

// bf16 bit pattern of x, rounded to nearest even (x finite)
short bf16_rne(double x) {
  const float f = (float)x;
  uint32_t u;
  std::memcpy(&u, &f, sizeof u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(uint16_t)(u >> 16);
}
double bf16_to_double(short b) {
  const uint32_t u = (uint32_t)(uint16_t)b << 16;
  float f;
  std::memcpy(&f, &u, sizeof f);
  return f;
}

// Three bf16 planes of an n x n block: x ~ x0 + x1 + x2 with x0 = bf16(x),
// x1 = bf16(x - x0), x2 = bf16(x - x0 - x1), residuals taken in FP64.
std::vector<short> split3(const std::vector<double>& a, int n) {
  const size_t m = (size_t)n * n;
  std::vector<short> out(3 * std::max<size_t>(m, 1), 0);
  for (size_t i = 0; i < m; ++i) {
    double r = a[i];
    for (int s = 0; s < 3; ++s) {
      const short b = bf16_rne(r);
      out[s * m + i] = b;
      r -= bf16_to_double(b);
    }
  }
  return out;
}

// Three FP16 planes of 2^12 a (|a| <= 1 here), rounded to nearest even, with
// residuals taken in FP64.
std::vector<short> split3_f16(const std::vector<double>& a, int n) {
  const size_t m = (size_t)n * n;
  std::vector<short> out(3 * std::max<size_t>(m, 1), 0);
  for (size_t i = 0; i < m; ++i) {
    double r = a[i] * 4096.0;
    for (int s = 0; s < 3; ++s) {
      const _Float16 h = (_Float16)r;
      short b;
      std::memcpy(&b, &h, sizeof b);
      out[s * m + i] = b;
      r -= (double)h;
    }
  }
  return out;
}

size_t elem_size(int dtype) { return dtype == KX_F64 ? sizeof(double) : sizeof(float); }

bool all_dirichlet(const kx_grid* g) {
  return g->bc[0] == KX_BC_DIRICHLET && g->bc[1] == KX_BC_DIRICHLET && g->bc[2] == KX_BC_DIRICHLET;
}

bool all_periodic(const kx_grid* g) {
  return g->bc[0] == KX_BC_PERIODIC && g->bc[1] == KX_BC_PERIODIC && g->bc[2] == KX_BC_PERIODIC;
}

double lam_min_host(const kx_grid* g) {
  // lam_host is ascending per axis
  return g->lam_host[0][0] + g->lam_host[1][0] + g->lam_host[2][0];
}

kx_status check_kernel_args(const kx_grid* g, int kernel, double omega) {
  if (kernel != KX_KERNEL_COULOMB && kernel != KX_KERNEL_ERFC) return KX_ERR_INVALID_ARG;
  if (kernel == KX_KERNEL_ERFC && !(std::isfinite(omega) && omega > 0.0)) return KX_ERR_INVALID_ARG;
  if (kernel == KX_KERNEL_COULOMB && !g->zero.on &&
      (all_periodic(g) || !(lam_min_host(g) > 0.0)))
    return KX_ERR_SINGULAR;
  return KX_OK;
}

kx_status check_types(const kx_grid* g, int dtype, int prec) {
  if (dtype != KX_F64 && dtype != KX_F32) return KX_ERR_INVALID_ARG;
  if (prec < KX_PREC_FP64 || prec > KX_PREC_MIXED) return KX_ERR_INVALID_ARG;
  if (prec == KX_PREC_MIXED)  // FP64 forward pass, split inverse pass
    return g->plan_d.fwd.ok && g->plan_s.inv.ok ? KX_OK : KX_ERR_UNSUPPORTED;
  // BF16X3 and FP16X3 share the split kernels' launch shapes
  const Plan& p = prec == KX_PREC_FP64 ? g->plan_d : (prec == KX_PREC_FP32 ? g->plan_f : g->plan_s);
  if (!p.fwd.ok || !p.inv.ok) return KX_ERR_UNSUPPORTED;
  return KX_OK;
}

// True while work on stream s is being recorded into a graph.
bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return cs == hipStreamCaptureStatusActive;
}

// f(lam1_a + lam2_b + lam3_c) for the requested kernel, written by a kernel
// into the handle's table (every application writes it, so that work
// recorded into a graph carries its own table).
// With KX_CHECK_FINITE set: KX_ERR_NUMERIC if any of the n values at p is
// NaN or infinite.  Synchronises the stream.
kx_status check_finite(kx_grid* g, const void* p, int storage, long long n) {
  if (!(g->checks & KX_CHECK_FINITE) || n <= 0) return KX_OK;
  KX_HIP(launch_nonfinite(p, storage, n, g->dFlag, g->stream));
  unsigned v = 0;
  KX_HIP(hipMemcpyAsync(&v, g->dFlag, sizeof(v), hipMemcpyDeviceToHost, g->stream));
  KX_HIP(hipStreamSynchronize(g->stream));
  return v ? KX_ERR_NUMERIC : KX_OK;
}
// checks on a stream that is being recorded would synchronise it
bool checks_block_capture(const kx_grid* g) {
  return (g->checks & KX_CHECK_FINITE) && stream_capturing(g->stream);
}

hipError_t fill_ftable(kx_grid* g, int kernel, double omega, hipStream_t s) {
  const double om = (kernel == KX_KERNEL_ERFC) ? omega : 0.0;
  const double* le[3] = {g->dLamE[0], g->dLamE[1], g->dLamE[2]};
  const double* lo[3] = {g->dLamO[0], g->dLamO[1], g->dLamO[2]};
  return launch_ftable(le, lo, g->geom, kernel, om, g->dF, s, g->zero);
}

// Bytes of one slot of the intermediate for precision prec.
size_t t_bytes(const Geom& G, int prec) {
  const bool dbl = prec == KX_PREC_FP64 || prec == KX_PREC_MIXED;
  return (dbl ? sizeof(double) : sizeof(float)) * (size_t)G.slot;
}

// Grow the handle's per-launch buffers to `slots` items: T (8-byte values, so
// that every precision fits), the energy partials, the field items, and, when
// asked, the mixed path's FP32 copy and the split-FP16 result maxima.  The
// padded rows of the intermediates are never written by the transform kernels
// and are cleared here, by a kernel.  May synchronise the stream.
kx_status reserve_slots(kx_grid* g, int slots, bool t2, bool aux16) {
  Work& w = g->ws;
  const Geom& G = g->geom;
  const bool grow_t = slots > w.slots;
  const bool grow_t2 = t2 && (grow_t || !w.T2);
  const bool grow_aux = aux16 && (grow_t || !w.tmax);
  if (!grow_t && !grow_t2 && !grow_aux) return KX_OK;
  // the previous buffers may still be in use by queued work
  KX_HIP(hipStreamSynchronize(g->stream));
  ++g->gen;
  const int ns = std::max(slots, w.slots);
  if (grow_t) {
    dev_free(w.T);
    dev_free(w.epart);
    dev_free(w.fitems);
    dev_free(w.mpart);
    dev_free(w.mmom);
    dev_free(w.fields);
    w.T = nullptr;
    w.epart = nullptr;
    w.fitems = nullptr;
    w.mpart = nullptr;
    w.mmom = nullptr;
    w.fields = nullptr;
    w.slots = 0;
    const size_t tb = sizeof(double) * (size_t)G.slot * ns;
    kx_status st = dev_alloc(&w.T, tb);
    if (st != KX_OK) return st;
    KX_HIP(launch_zero(w.T, tb, g->stream));
    const size_t nstrips = (size_t)(G.slab / kTile);
    st = dev_alloc((void**)&w.epart, sizeof(double) * nstrips * ns);
    if (st != KX_OK) return st;
    st = dev_alloc((void**)&w.fitems, sizeof(Item) * ns);
    if (st != KX_OK) return st;
    KX_HIP(launch_field_items(ns, w.fitems, g->stream));
    if (all_dirichlet(g)) {  // multipole boundary values of batches of fields
      const size_t K = (size_t)(kMaxMultipoleL + 1) * (kMaxMultipoleL + 1);
      st = dev_alloc((void**)&w.mpart, sizeof(double) * K * multipole_groups(G.N) * ns);
      if (st != KX_OK) return st;
      st = dev_alloc((void**)&w.mmom, sizeof(double) * K * ns);
      if (st != KX_OK) return st;
      st = dev_alloc((void**)&w.fields, sizeof(double) * (size_t)G.N * ns);
      if (st != KX_OK) return st;
    }
    w.slots = ns;
    w.tbytes = sizeof(double) * (size_t)G.slot;
    kx_logf("workspace: %d launch slots, %.1f MB of intermediates", ns, tb / 1e6);
  }
  if (grow_t2 || (w.T2 && grow_t)) {
    dev_free(w.T2);
    w.T2 = nullptr;
    const size_t b = sizeof(float) * (size_t)G.slot * ns;
    kx_status st = dev_alloc((void**)&w.T2, b);
    if (st != KX_OK) return st;
    KX_HIP(launch_zero(w.T2, b, g->stream));
  }
  if (grow_aux || (w.tmax && grow_t)) {
    dev_free(w.tmax);
    w.tmax = nullptr;
    kx_status st = dev_alloc((void**)&w.tmax, sizeof(unsigned) * ns);
    if (st != KX_OK) return st;
  }
  return KX_OK;
}

// grow a device array to n elements of `size` bytes (contents not kept)
template <class T>
kx_status grow(kx_grid* g, T** p, long long* cap, long long n) {
  if (n <= *cap) return KX_OK;
  KX_HIP(hipStreamSynchronize(g->stream));
  ++g->gen;
  dev_free(*p);
  *p = nullptr;
  *cap = 0;
  kx_status st = dev_alloc((void**)p, sizeof(T) * (size_t)std::max<long long>(n, 1));
  if (st != KX_OK) return st;
  *cap = n;
  return KX_OK;
}

// Every buffer an exchange application on up to norb orbitals (or, with
// norb == 0, batches of fields) in precision prec on storage dtype needs.
kx_status reserve(kx_grid* g, int norb, int prec, int dtype) {
  const int slots = norb > 0 ? std::min(g->max_slots, norb) : g->max_slots;
  kx_status st = reserve_slots(g, slots, prec == KX_PREC_MIXED, prec == KX_PREC_FP16X3);
  if (st != KX_OK) return st;
  Work& w = g->ws;
  if (prec == KX_PREC_FP16X3) {  // one scale per orbital, or per field of a launch
    long long cap = w.omax_cap;
    st = grow(g, &w.omax, &cap, std::max(norb, w.slots));
    if (st != KX_OK) return st;
    w.omax_cap = (int)cap;
  }
  if (norb == 0) return KX_OK;
  const long long npairs = (long long)norb * (norb + 1) / 2;
  long long cap = w.items_cap;
  st = grow(g, &w.items, &cap, npairs);
  if (st != KX_OK) return st;
  w.items_cap = cap;
  cap = w.pairE_cap;
  st = grow(g, &w.pairE, &cap, npairs);
  if (st != KX_OK) return st;
  w.pairE_cap = cap;
  cap = w.occ_cap;
  st = grow(g, &w.occ, &cap, norb);
  if (st != KX_OK) return st;
  w.occ_cap = (int)cap;
  if (norb <= kXTileMaxOrb && prec != KX_PREC_FP16X3) {  // the two-stage exchange's potentials
    st = grow(g, &w.phi, &w.phi_cap, (long long)kXTile * kXTile * g->geom.N);
    if (st != KX_OK) return st;
  }
  if (all_dirichlet(g)) {  // the isolated-system exchange's energy partials
    st = grow(g, &w.dpart, &w.dpart_cap, (long long)norb * vx_energy_parts());
    if (st != KX_OK) return st;
  }
  if (prec != KX_PREC_FP64 && dtype == KX_F64) {
    const long long nel = (long long)norb * g->geom.N;
    long long c1 = (long long)w.work32_cap, c2 = (long long)w.work32_cap;
    st = grow(g, &w.psi32, &c1, nel);
    if (st != KX_OK) return st;
    st = grow(g, &w.vx32, &c2, nel);
    if (st != KX_OK) return st;
    w.work32_cap = (size_t)std::min(c1, c2);
  }
  return KX_OK;
}

void free_work(Work& w) {
  dev_free(w.phi);
  dev_free(w.mpart);
  dev_free(w.mmom);
  dev_free(w.fields);
  dev_free(w.dpart);
  dev_free(w.T);
  dev_free(w.T2);
  dev_free(w.epart);
  dev_free(w.tmax);
  dev_free(w.fitems);
  dev_free(w.items);
  dev_free(w.pairE);
  dev_free(w.occ);
  dev_free(w.omax);
  dev_free(w.psi32);
  dev_free(w.vx32);
  w = Work();
}

// ---- the fixed scratch array of kx_apply_exchange_noalloc
// One per device, allocated with the code object and held until the process
// ends.  Host code must not pass its name to a kernel: the name is a host-side
// stand-in, not a device address.  The device address, per device, comes from
// hipGetSymbolAddress at set-up.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[KX_SCRATCH_BYTES];

namespace {

// Look up this device's copy of the scratch array, once per device (the
// device current at the call).
kx_status scratch_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return KX_ERR_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return KX_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return KX_ERR_DEVICE;
  }
  g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  return KX_OK;
}

// The buffers of one exchange application on norb orbitals in precision prec,
// carved out of the handle's device's scratch array: the pair schedule, pair
// energies, occupations and FP16 scales first, then as many launch slots (T,
// the mixed path's T2, energy partials, FP16 result maxima) as fit, up to the
// handle's batch size.  No FP32 working copies: the kernels read the caller's
// storage.  KX_ERR_OUT_OF_MEMORY if not even one slot fits.
kx_status carve_scratch(const kx_grid* g, int norb, int prec, Work& w) {
  w = Work();
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g->device >= 0 && g->device < kMaxDevices) base = g_scratch_ptr[g->device];
  }
  if (!base) return KX_ERR_STATE;
  if (norb == 0) return KX_OK;
  const Geom& G = g->geom;
  const size_t cap = KX_SCRATCH_BYTES;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) / 256 * 256;
    return base + o;
  };
  const long long npairs = (long long)norb * (norb + 1) / 2;
  const bool mixed = prec == KX_PREC_MIXED, h16 = prec == KX_PREC_FP16X3;
  const size_t fixed = (sizeof(Item) + sizeof(double)) * (size_t)npairs + sizeof(double) * norb +
                       (h16 ? sizeof(float) * norb : 0) + 4 * 256;
  const size_t nstrips = (size_t)(G.slab / kTile);
  const size_t tb = t_bytes(G, prec);
  const size_t per_slot =
      tb + (mixed ? sizeof(float) * (size_t)G.slot : 0) + sizeof(double) * nstrips + (h16 ? 4 : 0);
  if (fixed >= cap) return KX_ERR_OUT_OF_MEMORY;
  long long slots = (long long)((cap - fixed - 4 * 256) / per_slot);
  slots = std::min<long long>(slots, std::min(g->batch_cap, norb));
  if (slots < 1) return KX_ERR_OUT_OF_MEMORY;
  w.items = reinterpret_cast<Item*>(take(sizeof(Item) * npairs));
  w.items_cap = npairs;
  w.pairE = reinterpret_cast<double*>(take(sizeof(double) * npairs));
  w.pairE_cap = npairs;
  w.occ = reinterpret_cast<double*>(take(sizeof(double) * norb));
  w.occ_cap = norb;
  if (h16) {
    w.omax = reinterpret_cast<float*>(take(sizeof(float) * norb));
    w.omax_cap = norb;
  }
  w.T = take(tb * slots);
  w.tbytes = tb;
  if (mixed) w.T2 = reinterpret_cast<float*>(take(sizeof(float) * G.slot * slots));
  w.epart = reinterpret_cast<double*>(take(sizeof(double) * nstrips * slots));
  if (h16) w.tmax = reinterpret_cast<unsigned*>(take(sizeof(unsigned) * slots));
  w.slots = (int)slots;
  return off <= cap ? KX_OK : KX_ERR_OUT_OF_MEMORY;
}

// Bracket one kernel launch with timing events when profiling is on.
template <class F>
hipError_t timed(kx_grid* g, hipStream_t s, int kind, F&& launch) {
  if (!g->prof_on || g->capturing || !((g->prof_mask >> kind) & 1)) return launch();
  const size_t k = g->prof_kind.size();
  if (g->recording && g->prof_ev.size() < 2 * (k + 1)) return launch();
  while (g->prof_ev.size() < 2 * (k + 1)) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) return hipErrorOutOfMemory;
    g->prof_ev.push_back(ev);
  }
  hipError_t e = hipEventRecord(g->prof_ev[2 * k], s);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(g->prof_ev[2 * k + 1], s);
  g->prof_kind.push_back(kind);
  return e;
}

// One batch of nb items through the three transform passes (and, for the
// exchange, the per-pair energy reduction), in the arithmetic of prec, in the
// buffers of w.  src (the forward pass input) has storage src_dtype; psi and
// dst (the inverse pass) have storage dtype.
hipError_t run_batch(kx_grid* g, const Work& w, hipStream_t st, int mode, int prec, int src_dtype,
                     const void* src, const Item* it, int nb, int dtype, const void* psi,
                     const double* occ, void* dst, int norb, double dV) {
  const Geom& G = g->geom;
  double* epart = mode == 1 ? w.epart : nullptr;
  const int nstrips = (int)(G.slab / kTile);
  hipError_t e;
  if (prec == KX_PREC_MIXED) {
    // forward, f scaling and energies in FP64; the pencil's result rounded
    // into the FP32 intermediate; split-BF16 inverse pass
    const EigR<double> E = eig_of(g);
    double* T = (double*)w.T;
    e = timed(g, st, KX_PHASE_FORWARD, [&] {
      return launch_forward_d(src_dtype, mode, G, g->plan_d.fwd, E, src, it, nb, T, st);
    });
    if (e != hipSuccess) return e;
    e = timed(g, st, KX_PHASE_PENCIL, [&] {
      return launch_pencil_d(G, g->plan_d.pen, E, g->dF, nb, T, epart, st, w.T2);
    });
    if (e != hipSuccess) return e;
    if (mode == 1) {
      e = timed(g, st, KX_PHASE_ENERGY, [&] {
        return launch_pair_energy(epart, nstrips, it, nb, norb, dV, w.pairE, st);
      });
      if (e != hipSuccess) return e;
    }
    return timed(g, st, KX_PHASE_INVERSE, [&] {
      return launch_inverse_s(dtype, mode, G, g->plan_s.inv, eigs_of(g), w.T2, it, nb, psi, occ,
                              dst, st);
    });
  }
  if (prec == KX_PREC_FP64) {
    const EigR<double> E = eig_of(g);
    double* T = (double*)w.T;
    e = timed(g, st, KX_PHASE_FORWARD, [&] {
      return launch_forward_d(src_dtype, mode, G, g->plan_d.fwd, E, src, it, nb, T, st);
    });
    if (e != hipSuccess) return e;
    e = timed(g, st, KX_PHASE_PENCIL, [&] {
      return launch_pencil_d(G, g->plan_d.pen, E, g->dF, nb, T, epart, st);
    });
    if (e != hipSuccess) return e;
    if (mode == 1) {
      e = timed(g, st, KX_PHASE_ENERGY, [&] {
        return launch_pair_energy(epart, nstrips, it, nb, norb, dV, w.pairE, st);
      });
      if (e != hipSuccess) return e;
    }
    return timed(g, st, KX_PHASE_INVERSE, [&] {
      return launch_inverse_d(dtype, mode, G, g->plan_d.inv, E, T, it, nb, psi, occ, dst, st);
    });
  }
  if (prec == KX_PREC_BF16X3 || prec == KX_PREC_FP16X3) {
    const bool h16 = prec == KX_PREC_FP16X3;
    const EigS E = h16 ? eigh_of(g) : eigs_of(g);
    SplitAux aux;
    if (h16) {  // the source maxima were computed before the batches
      aux.h16 = 1;
      aux.omax = w.omax;
      aux.tmax = w.tmax;
      e = launch_zero(w.tmax, sizeof(unsigned) * nb, st);
      if (e != hipSuccess) return e;
    }
    float* T = (float*)w.T;
    e = timed(g, st, KX_PHASE_FORWARD, [&] {
      return launch_forward_s(src_dtype, mode, G, g->plan_s.fwd, E, src, it, nb, T, st, aux);
    });
    if (e != hipSuccess) return e;
    e = timed(g, st, KX_PHASE_PENCIL, [&] {
      return launch_pencil_s(G, g->plan_s.pen, E, g->dF, nb, T, epart, st, aux);
    });
    if (e != hipSuccess) return e;
    if (mode == 1) {
      e = timed(g, st, KX_PHASE_ENERGY, [&] {
        return launch_pair_energy(epart, nstrips, it, nb, norb, dV, w.pairE, st);
      });
      if (e != hipSuccess) return e;
    }
    return timed(g, st, KX_PHASE_INVERSE, [&] {
      return launch_inverse_s(dtype, mode, G, g->plan_s.inv, E, T, it, nb, psi, occ, dst, st,
                              aux);
    });
  }
  const EigR<float> E = eigf_of(g);
  float* T = (float*)w.T;
  e = timed(g, st, KX_PHASE_FORWARD, [&] {
    return launch_forward_f(src_dtype, mode, G, g->plan_f.fwd, E, src, it, nb, T, st);
  });
  if (e != hipSuccess) return e;
  e = timed(g, st, KX_PHASE_PENCIL, [&] {
    return launch_pencil_f(G, g->plan_f.pen, E, g->dF, nb, T, epart, st);
  });
  if (e != hipSuccess) return e;
  if (mode == 1) {
    e = timed(g, st, KX_PHASE_ENERGY, [&] {
      return launch_pair_energy(epart, nstrips, it, nb, norb, dV, w.pairE, st);
    });
    if (e != hipSuccess) return e;
  }
  return timed(g, st, KX_PHASE_INVERSE, [&] {
    return launch_inverse_f(dtype, mode, G, g->plan_f.inv, E, T, it, nb, psi, occ, dst, st);
  });
}

// One exchange application, resolved against a set of buffers.
struct XPlan {
  int kernel = 0, norb = 0, prec = 0, dtype = 0, dtype_w = 0;
  double omega = 0.0, dV = 0.0;
  bool narrow = false;  // reduced precision on FP64 storage: FP32 working copies
  const void* psi = nullptr;
  void* vx = nullptr;
  const void* psi_w = nullptr;
  void* vx_w = nullptr;
  size_t nel = 0;
  std::vector<double> occ;      // the occupations, sent to the device as kernel arguments
  std::vector<int> offsets;     // batch offsets into the pair schedule
};

// Validate the arguments of one exchange application and check that w holds
// everything it needs.  Touches no device state.
kx_status plan_exchange(const kx_grid* g, const Work& w, int kernel, double omega, int norb,
                        int dtype, const void* psi_dev, const double* occ_host, void* vxpsi_dev,
                        int prec, XPlan& xp) {
  if (!g || norb < 0 || norb > 65535) return KX_ERR_INVALID_ARG;
  if (g->nonorth) return KX_ERR_UNSUPPORTED;  // mixed derivatives couple the real modes
  kx_status st = check_kernel_args(g, kernel, omega);
  if (st != KX_OK) return st;
  st = check_types(g, dtype, prec);
  if (st != KX_OK) return st;
  if (norb > 0 && (!psi_dev || !vxpsi_dev || !occ_host)) return KX_ERR_INVALID_ARG;
  if (psi_dev && psi_dev == vxpsi_dev) return KX_ERR_INVALID_ARG;
  if ((double)norb * (double)g->geom.N > 4.0e18) return KX_ERR_INVALID_ARG;
  for (int i = 0; i < norb; ++i)
    if (!std::isfinite(occ_host[i])) return KX_ERR_INVALID_ARG;
  const long long npairs = (long long)norb * (norb + 1) / 2;
  xp = XPlan();
  xp.kernel = kernel;
  xp.omega = omega;
  xp.norb = norb;
  xp.prec = prec;
  xp.dtype = xp.dtype_w = dtype;
  xp.psi = xp.psi_w = psi_dev;
  xp.vx = xp.vx_w = vxpsi_dev;
  xp.dV = g->h[0] * g->h[1] * g->h[2];
  if (norb == 0) return KX_OK;
  if (w.slots < 1 || w.items_cap < npairs || w.pairE_cap < npairs || w.occ_cap < norb)
    return KX_ERR_STATE;
  if (prec == KX_PREC_MIXED && !w.T2) return KX_ERR_STATE;
  if (prec == KX_PREC_FP16X3 && (!w.tmax || w.omax_cap < norb)) return KX_ERR_STATE;
  xp.occ.assign(occ_host, occ_host + norb);
  schedule_offsets(norb, std::min(g->batch_cap, w.slots), xp.offsets);
  // Reduced precision on FP64 storage: the orbitals are rounded to FP32 once
  // and Vx psi is accumulated in FP32, then widened into the output; the
  // per-pair passes then move half the bytes.
  xp.nel = (size_t)norb * g->geom.N;
  xp.narrow = prec != KX_PREC_FP64 && dtype == KX_F64 && xp.nel <= w.work32_cap &&
              (reinterpret_cast<uintptr_t>(psi_dev) % 16) == 0 &&
              (reinterpret_cast<uintptr_t>(vxpsi_dev) % 16) == 0;
  if (xp.narrow) {
    xp.psi_w = w.psi32;
    xp.vx_w = w.vx32;
    xp.dtype_w = KX_F32;
  }
  return KX_OK;
}

// The two-stage exchange: per tile of kXTile x kXTile orbital pairs the
// forward pass (pair products), the pencil with the pair energies, the inverse
// pass writing the tile's potentials phi_ij, and one accumulation kernel that
// applies them to Vx psi, reading and writing each orbital of the tile once
// (the fused inverse pass read-modify-writes two orbitals per pair).
// FP64 takes it on FP64 storage, where the fused pass's orbital traffic (48 of
// its 56 bytes per pair and point) is what bounds it; with FP32 storage that
// share is 24 of 32 bytes and the fused pass stays faster (measured at
// 144^3).  The mixed, FP32 and BF16x3 paths, with FP32 potentials, take it
// everywhere (equal or faster at 96^3 and 144^3); FP16x3 keeps the fused pass
// (its scales follow the fused pass's items).
bool tiled_exchange(const kx_grid* g, const XPlan& xp, const Work& w) {
  const Geom& G = g->geom;
  if (!w.phi || xp.norb > kXTileMaxOrb || w.phi_cap < (long long)kXTile * kXTile * G.N ||
      w.slots < 1)
    return false;
  if (xp.prec == KX_PREC_FP64) return xp.dtype == KX_F64;
  return xp.prec == KX_PREC_MIXED || xp.prec == KX_PREC_FP32 || xp.prec == KX_PREC_BF16X3;
}

// the transforms of one launch of the two-stage exchange: pair products,
// forward modes, the pencil with its pair energies and the inverse modes into
// the potentials phi (FP64 for KX_PREC_FP64, FP32 otherwise)
hipError_t tiled_transforms(kx_grid* g, const XPlan& xp, const Work& w, hipStream_t s,
                            const Item* it, int nb, void* phi) {
  const Geom& G = g->geom;
  const int nstrips = (int)(G.slab / kTile);
  auto energy = [&] {
    return timed(g, s, KX_PHASE_ENERGY, [&] {
      return launch_pair_energy(w.epart, nstrips, it, nb, xp.norb, xp.dV, w.pairE, s);
    });
  };
  hipError_t e = hipSuccess;
  if (xp.prec == KX_PREC_FP64 || xp.prec == KX_PREC_MIXED) {
    const EigR<double> E = eig_of(g);
    double* T = (double*)w.T;
    const bool mixed = xp.prec == KX_PREC_MIXED;
    e = timed(g, s, KX_PHASE_FORWARD, [&] {
      return launch_forward_d(xp.dtype, 1, G, g->plan_d.fwd, E, xp.psi, it, nb, T, s);
    });
    if (e == hipSuccess)
      e = timed(g, s, KX_PHASE_PENCIL, [&] {
        return launch_pencil_d(G, g->plan_d.pen, E, g->dF, nb, T, w.epart, s,
                               mixed ? w.T2 : nullptr);
      });
    if (e == hipSuccess) e = energy();
    if (e == hipSuccess)
      e = timed(g, s, KX_PHASE_INVERSE, [&] {
        return mixed ? launch_inverse_s(KX_F32, 0, G, g->plan_s.inv, eigs_of(g), w.T2, w.fitems,
                                        nb, nullptr, nullptr, phi, s)
                     : launch_inverse_d(KX_F64, 0, G, g->plan_d.inv, E, T, w.fitems, nb, nullptr,
                                        nullptr, phi, s);
      });
    return e;
  }
  float* T = (float*)w.T;
  if (xp.prec == KX_PREC_FP32) {
    const EigR<float> E = eigf_of(g);
    e = timed(g, s, KX_PHASE_FORWARD, [&] {
      return launch_forward_f(xp.dtype_w, 1, G, g->plan_f.fwd, E, xp.psi_w, it, nb, T, s);
    });
    if (e == hipSuccess)
      e = timed(g, s, KX_PHASE_PENCIL, [&] {
        return launch_pencil_f(G, g->plan_f.pen, E, g->dF, nb, T, w.epart, s);
      });
    if (e == hipSuccess) e = energy();
    if (e == hipSuccess)
      e = timed(g, s, KX_PHASE_INVERSE, [&] {
        return launch_inverse_f(KX_F32, 0, G, g->plan_f.inv, E, T, w.fitems, nb, nullptr,
                                nullptr, phi, s);
      });
    return e;
  }
  const EigS E = eigs_of(g);  // split BF16
  e = timed(g, s, KX_PHASE_FORWARD, [&] {
    return launch_forward_s(xp.dtype_w, 1, G, g->plan_s.fwd, E, xp.psi_w, it, nb, T, s);
  });
  if (e == hipSuccess)
    e = timed(g, s, KX_PHASE_PENCIL, [&] {
      return launch_pencil_s(G, g->plan_s.pen, E, g->dF, nb, T, w.epart, s);
    });
  if (e == hipSuccess) e = energy();
  if (e == hipSuccess)
    e = timed(g, s, KX_PHASE_INVERSE, [&] {
      return launch_inverse_s(KX_F32, 0, G, g->plan_s.inv, E, T, w.fitems, nb, nullptr, nullptr,
                              phi, s);
    });
  return e;
}

hipError_t enqueue_exchange_tiled(kx_grid* g, const XPlan& xp, const Work& w, hipStream_t s) {
  const Geom& G = g->geom;
  const int norb = xp.norb;
  const int phi_storage = xp.prec == KX_PREC_FP64 ? KX_F64 : KX_F32;
  const size_t phi_field = elem_size(phi_storage) * (size_t)G.N;
  hipError_t e = fill_ftable(g, xp.kernel, xp.omega, s);
  if (e == hipSuccess) e = launch_tile_schedule(norb, w.items, s);
  if (e == hipSuccess) e = launch_put_doubles(xp.occ.data(), norb, w.occ, s);
  if (e == hipSuccess && xp.narrow)
    e = launch_narrow((const double*)xp.psi, w.psi32, (long long)xp.nel, s);
  if (e == hipSuccess) e = launch_zero(xp.vx_w, elem_size(xp.dtype_w) * xp.nel, s);
  const int nbk = (norb + kXTile - 1) / kXTile;
  long long off = 0;
  for (int a = 0; a < nbk && e == hipSuccess; ++a)
    for (int b = a; b < nbk && e == hipSuccess; ++b) {
      const int npt = xtile_pairs(a, b, norb);
      // the tile's pairs through the transforms in launches of up to `slots`
      for (int p0 = 0; p0 < npt && e == hipSuccess; p0 += w.slots) {
        const int nb = std::min(w.slots, npt - p0);
        e = tiled_transforms(g, xp, w, s, w.items + off + p0, nb,
                             static_cast<char*>(static_cast<void*>(w.phi)) + phi_field * p0);
      }
      off += npt;
      if (e == hipSuccess)
        e = timed(g, s, KX_PHASE_ACCUM, [&] {
          return launch_tile_accumulate(xp.dtype_w, phi_storage, w.phi, a, b, norb, G.N, xp.psi_w,
                                        w.occ, xp.vx_w, s);
        });
    }
  if (e == hipSuccess && xp.narrow) e = launch_widen(w.vx32, (double*)xp.vx, (long long)xp.nel, s);
  if (e != hipSuccess) return e;
  return timed(g, s, KX_PHASE_ENERGY, [&] {
    return launch_exchange_energy(w.pairE, w.occ, norb, g->dEx, s);
  });
}

// The device work of one planned exchange application on stream s: kernels
// only (no allocation, host transfer, memset or synchronisation), so it can
// be recorded into a graph.  The f table, the pair schedule and the
// occupations are written by kernels first.
hipError_t enqueue_exchange(kx_grid* g, const XPlan& xp, const Work& w, hipStream_t s) {
  if (xp.norb == 0) return launch_zero(g->dEx, sizeof(double), s);
  if (tiled_exchange(g, xp, w)) return enqueue_exchange_tiled(g, xp, w, s);
  hipError_t e = fill_ftable(g, xp.kernel, xp.omega, s);
  if (e == hipSuccess) e = launch_schedule(xp.norb, w.items, s);
  if (e == hipSuccess) e = launch_put_doubles(xp.occ.data(), xp.norb, w.occ, s);
  if (e != hipSuccess) return e;
  if (xp.narrow) {
    e = launch_narrow((const double*)xp.psi, w.psi32, (long long)xp.nel, s);
    if (e != hipSuccess) return e;
  }
  e = launch_zero(xp.vx_w, elem_size(xp.dtype_w) * xp.nel, s);
  if (e != hipSuccess) return e;
  if (xp.prec == KX_PREC_FP16X3) {  // the orbitals' largest magnitudes set the FP16 scales
    e = launch_absmax(xp.psi_w, xp.dtype_w, (long long)g->geom.N, xp.norb, w.omax, s);
    if (e != hipSuccess) return e;
  }
  // the mixed path's FP64 forward pass reads the caller's orbitals
  const bool mixed = xp.prec == KX_PREC_MIXED;
  for (size_t b = 0; b + 1 < xp.offsets.size(); ++b) {
    const int o0 = xp.offsets[b], nb = xp.offsets[b + 1] - o0;
    if (nb <= 0) continue;
    e = run_batch(g, w, s, 1, xp.prec, mixed ? xp.dtype : xp.dtype_w, mixed ? xp.psi : xp.psi_w,
                  w.items + o0, nb, xp.dtype_w, xp.psi_w, w.occ, xp.vx_w, xp.norb, xp.dV);
    if (e != hipSuccess) return e;
  }
  if (xp.narrow) {
    e = launch_widen(w.vx32, (double*)xp.vx, (long long)xp.nel, s);
    if (e != hipSuccess) return e;
  }
  return timed(g, s, KX_PHASE_ENERGY, [&] {
    return launch_exchange_energy(w.pairE, w.occ, xp.norb, g->dEx, s);
  });
}

// Drop the recorded multi-system graph (and, with all, its streams/events).
void release_batch_graph(kx_grid* g, bool all) {
  auto& b = g->batch;
  if (b.origin) (void)hipStreamSynchronize(b.origin);
  if (b.exec) (void)hipGraphExecDestroy(b.exec);
  if (b.graph) (void)hipGraphDestroy(b.graph);
  b.exec = nullptr;
  b.graph = nullptr;
  b.key.clear();
  if (!all) return;
  for (hipStream_t s : b.branch) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b.join) (void)hipEventDestroy(e);
  if (b.fork) (void)hipEventDestroy(b.fork);
  if (b.origin) (void)hipStreamDestroy(b.origin);
  b.branch.clear();
  b.join.clear();
  b.fork = nullptr;
  b.origin = nullptr;
}

// ---- Brillouin-zone sampling (Sec. II)

// The coupled mode of every folded eigenvector under a Bloch phase, per
// periodic axis: the real part of V^T M(theta0) V must be diagonal and its
// imaginary part must couple each mode to at most one mode of the other
// parity (theta0 = 0.9, a generic phase).  Built once per handle from the
// device blocks; synchronises.  KX_ERR_NUMERIC if the structure is not found.
kx_status bloch_map(kx_grid* g) {
  auto& B = g->bl;
  if (B.mapped) return KX_OK;
  const Geom& G = g->geom;
  const int ns[3] = {G.n1, G.n2, G.n3}, mes[3] = {G.me1, G.me2, G.me3},
            mos[3] = {G.mo1, G.mo2, G.mo3}, pes[3] = {G.pe1, G.pe2, G.pe3},
            pos[3] = {G.po1, G.po2, G.po3};
  const int pmax = std::max(G.p1, std::max(G.p2, G.p3));
  std::vector<int> part((size_t)3 * pmax, -1);
  double w[kMaxStencil + 1];
  fd_weights_closed_form(g->order, w);
  const int m = g->order / 2;
  for (int a = 0; a < 3; ++a) {
    if (g->bc[a] != KX_BC_PERIODIC) continue;
    const int n = ns[a], me = mes[a], mo = mos[a], pe = pes[a], po = pos[a];
    std::vector<double> VE((size_t)pe * pe), VO((size_t)po * po);
    KX_HIP(hipStreamSynchronize(g->stream));
    KX_HIP(hipMemcpy(VE.data(), g->dVE[a], sizeof(double) * VE.size(), hipMemcpyDeviceToHost));
    if (po > 0)
      KX_HIP(hipMemcpy(VO.data(), g->dVO[a], sizeof(double) * VO.size(), hipMemcpyDeviceToHost));
    // full vectors of the valid blocked indices
    std::vector<int> ids;
    std::vector<std::vector<double>> v;
    for (int idx = 0; idx < pe + po; ++idx) {
      const bool even = idx < pe;
      if (even ? idx >= me : idx - pe >= mo) continue;
      std::vector<double> x(n, 0.0);
      for (int i = 0; i < n; ++i) {
        if (even) {
          const int j = i < me ? i : n - 1 - i;
          x[i] = VE[(size_t)j * pe + idx];
        } else if (i < mo) {
          x[i] = VO[(size_t)i * po + (idx - pe)];
        } else if (i >= n - mo) {
          x[i] = -VO[(size_t)(n - 1 - i) * po + (idx - pe)];
        }
      }
      ids.push_back(idx);
      v.push_back(std::move(x));
    }
    const double th = 0.9, h2 = g->h[a] * g->h[a];
    double scale = 0.0;
    std::vector<double> cr(2 * m + 1), ci(2 * m + 1);
    for (int p = -m; p <= m; ++p) {
      const double wp = w[std::abs(p)] / h2;
      cr[p + m] = -wp * std::cos(th * p / n);
      ci[p + m] = -wp * std::sin(th * p / n);
      scale += std::fabs(wp);
    }
    const double tol = 1e-10 * scale;
    const int nv = (int)ids.size();
    std::vector<double> R((size_t)nv * nv), I((size_t)nv * nv);
    std::vector<double> yr(n), yi(n);
    for (int c = 0; c < nv; ++c) {
      for (int i = 0; i < n; ++i) {
        double sr = 0.0, si = 0.0;
        for (int p = -m; p <= m; ++p) {
          const int j = ((i + p) % n + n) % n;
          sr += cr[p + m] * v[c][j];
          si += ci[p + m] * v[c][j];
        }
        yr[i] = sr;
        yi[i] = si;
      }
      for (int r = 0; r < nv; ++r) {
        double dr = 0.0, di = 0.0;
        for (int i = 0; i < n; ++i) {
          dr += v[r][i] * yr[i];
          di += v[r][i] * yi[i];
        }
        R[(size_t)r * nv + c] = dr;
        I[(size_t)r * nv + c] = di;
      }
    }
    std::vector<int> pr(nv, -1);
    for (int r = 0; r < nv; ++r) {
      int best = -1;
      for (int c = 0; c < nv; ++c) {
        if (c != r && std::fabs(R[(size_t)r * nv + c]) > tol) return KX_ERR_NUMERIC;
        if (std::fabs(I[(size_t)r * nv + c]) > tol) {
          if (best >= 0) return KX_ERR_NUMERIC;  // coupled to two modes
          best = c;
        }
      }
      pr[r] = best;
    }
    for (int r = 0; r < nv; ++r) {
      const int c = pr[r];
      if (c < 0) continue;
      if (pr[c] != r || (ids[r] < pe) == (ids[c] < pe)) return KX_ERR_NUMERIC;
      part[(size_t)a * pmax + ids[r]] = ids[c];
    }
  }
  // one coupling group per representative: the unpaired modes and the even
  // member of every pair
  std::vector<int> reps((size_t)3 * pmax, 0);
  for (int a = 0; a < 3; ++a) {
    int r = 0;
    for (int idx = 0; idx < pes[a] + pos[a]; ++idx) {
      const bool even = idx < pes[a];
      if (even ? idx >= mes[a] : idx - pes[a] >= mos[a]) continue;
      if (!even && part[(size_t)a * pmax + idx] >= 0) continue;
      reps[(size_t)a * pmax + r++] = idx;
    }
    B.nrep[a] = r;
  }
  kx_status st = dev_alloc((void**)&B.part, sizeof(int) * part.size());
  if (st != KX_OK) return st;
  KX_HIP(hipMemcpy(B.part, part.data(), sizeof(int) * part.size(), hipMemcpyHostToDevice));
  st = dev_alloc((void**)&B.reps, sizeof(int) * reps.size());
  if (st != KX_OK) return st;
  KX_HIP(hipMemcpy(B.reps, reps.data(), sizeof(int) * reps.size(), hipMemcpyHostToDevice));
  B.pmax = pmax;
  B.mapped = true;
  return KX_OK;
}

BlochAxes bloch_axes(const kx_grid* g) {
  const Geom& G = g->geom;
  BlochAxes B;
  const int ns[3] = {G.n1, G.n2, G.n3}, mes[3] = {G.me1, G.me2, G.me3},
            mos[3] = {G.mo1, G.mo2, G.mo3}, pes[3] = {G.pe1, G.pe2, G.pe3},
            pos[3] = {G.po1, G.po2, G.po3};
  for (int a = 0; a < 3; ++a) {
    BlochAxis& A = B.ax[a];
    A.n = ns[a];
    A.me = mes[a];
    A.mo = mos[a];
    A.pe = pes[a];
    A.po = pos[a];
    A.periodic = g->bc[a] == KX_BC_PERIODIC ? 1 : 0;
    A.h = g->h[a];
    A.VE = g->dVE[a];
    A.VO = g->dVO[a];
    A.lamE = g->dLamE[a];
    A.lamO = g->dLamO[a];
    A.part = g->bl.part + (size_t)a * g->bl.pmax;
  }
  for (int p = 0; p <= kMaxStencil; ++p) B.w[p] = B.d[p] = 0.0;
  fd_weights_closed_form(g->order, B.w);
  fd_weights_d1_closed_form(g->order, B.d);
  B.m = g->order / 2;
  B.nonorth = g->nonorth ? 1 : 0;
  B.zero = g->zero;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) B.gm[a][b] = g->cell_g[a][b];
  return B;
}

// The zero mode sits at rounding level; the smallest non-zero eigenvalue of
// a periodic axis is (2 pi / (n h))^2 and far above 1e-9 of the largest.
double zero_tolerance(const kx_grid* g) {
  double lam_max = 0.0;
  for (int a = 0; a < 3; ++a) lam_max += g->lam_host[a].back();
  double gs = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) gs += std::fabs(g->cell_g[a][b]);
  return 1e-9 * lam_max * std::max(1.0, gs);
}

// the volume element h1 h2 h3 |det E| of the cell
double cell_dV(const kx_grid* g) { return g->h[0] * g->h[1] * g->h[2] * g->cell_jac; }

RepMap bloch_reps(const kx_grid* g) {
  RepMap rm;
  for (int a = 0; a < 3; ++a) {
    rm.rep[a] = g->bl.reps + (size_t)a * g->bl.pmax;
    rm.R[a] = g->bl.nrep[a];
  }
  return rm;
}

// complex items (pairs, or fields) per launch of the Bloch path
int bloch_batch(const kx_grid* g) {
  return g->ws.slots / 2 >= kTileR * kTileC ? g->ws.slots / 2 : 0;
}
long long bloch_field_stride(const Geom& G) { return std::max(G.N, G.fsize); }

// One launch of nb complex items whose ramp-free real / imaginary parts are
// in Z (fields 2 t, 2 t + 1, stride N): forward modes 1, 2 and the forward
// mode-3 product into spectra (Z, stride fsize), the coupling (energy
// partials into epart), the inverse mode-3 product and the inverse modes 2, 1
// back into Z (stride N).
hipError_t bloch_solve(kx_grid* g, int kernel, double omega, const PairMap& pm, int nb,
                       hipStream_t s) {
  const Geom& G = g->geom;
  const EigR<double> E = eig_of(g);
  double* T = (double*)g->ws.T;
  double* Z = g->bl.Z;
  hipError_t e = timed(g, s, KX_PHASE_FORWARD, [&] {
    return launch_forward_d(KX_F64, 0, G, g->plan_d.fwd, E, Z, g->ws.fitems, 2 * nb, T, s);
  });
  if (e != hipSuccess) return e;
  e = timed(g, s, KX_PHASE_PENCIL, [&] {
    hipError_t r = launch_pencil_half(0, G, E, 2 * nb, T, Z, s);
    if (r == hipSuccess)
      r = launch_bloch_couple(bloch_axes(g), G, bloch_reps(g), g->bl.tab, g->bl.pmax, kernel,
                              omega, pm, nb, Z, g->bl.epart, s);
    if (r == hipSuccess) r = launch_pencil_half(1, G, E, 2 * nb, T, Z, s);
    return r;
  });
  if (e != hipSuccess) return e;
  return timed(g, s, KX_PHASE_INVERSE, [&] {
    return launch_inverse_d(KX_F64, 0, G, g->plan_d.inv, E, T, g->ws.fitems, 2 * nb, nullptr,
                            nullptr, Z, s);
  });
}

// the reserved Bloch buffers hold nk k-points of norb bands (nk == 0: fields)
bool bloch_reserved(const kx_grid* g, int nk, int norb) {
  const auto& B = g->bl;
  const Geom& G = g->geom;
  const int nb = bloch_batch(g);
  if (!B.mapped || nb < 1) return false;
  const int K = std::max(nk, 2);
  const long long M = (long long)nk * norb;
  return B.z_cap >= 2LL * nb * bloch_field_stride(G) &&
         B.epart_cap >= (long long)nb * bloch_couple_waves(bloch_reps(g)) &&
         B.tab_cap >= (long long)K * K * 3 * kBlochTab * B.pmax && B.kq_cap >= 3LL * K &&
         B.occw_cap >= M && B.u_cap >= 2 * M * G.N && B.w_cap >= 2 * M * G.N &&
         B.pairE_cap >= M * (M + 1) / 2;
}

}  // namespace

// ============================================================ C ABI
extern "C" {

const char* kx_status_string(int s) {
  switch (s) {
    case KX_OK: return "ok";
    case KX_ERR_INVALID_ARG: return "invalid argument";
    case KX_ERR_UNSUPPORTED: return "unsupported by the library";
    case KX_ERR_SINGULAR: return "singular: unscreened kernel with a zero eigenvalue";
    case KX_ERR_OUT_OF_MEMORY: return "out of memory";
    case KX_ERR_DEVICE: return "HIP runtime error";
    case KX_ERR_STATE: return "invalid state";
    case KX_ERR_NUMERIC: return "numerical failure";
    default: return "unknown status";
  }
}

kx_status kx_fd_weights(int fd_order, double* w_out) {
  if (!valid_order(fd_order) || !w_out) return KX_ERR_INVALID_ARG;
  fd_weights_closed_form(fd_order, w_out);
  return KX_OK;
}

kx_status kx_laplacian_1d(int n, double h, int fd_order, int bc, double* L_out) {
  if (n < 1 || n > kMaxN || !(std::isfinite(h) && h > 0.0) || !valid_order(fd_order) || !L_out ||
      (bc != KX_BC_DIRICHLET && bc != KX_BC_PERIODIC))
    return KX_ERR_INVALID_ARG;
  laplacian_1d(n, h, fd_order, bc, L_out);
  return KX_OK;
}

kx_status kx_pair_schedule(int norb, int max_batch, int* npairs_out, int* nbatches_out,
                           int* pairs_out, int* batch_offsets_out) {
  if (norb < 0 || norb > 65535 || !npairs_out || !nbatches_out) return KX_ERR_INVALID_ARG;
  std::vector<Item> pairs;
  std::vector<int> o2;
  schedule_pairs(norb, pairs);
  schedule_offsets(norb, max_batch, o2);
  *npairs_out = (int)pairs.size();
  *nbatches_out = (int)o2.size() - 1;
  if (pairs_out) {
    for (size_t k = 0; k < pairs.size(); ++k) {
      pairs_out[2 * k] = pairs[k].i;
      pairs_out[2 * k + 1] = pairs[k].j;
    }
  }
  if (batch_offsets_out)
    for (size_t b = 0; b < o2.size(); ++b) batch_offsets_out[b] = o2[b];
  return KX_OK;
}

kx_status kx_setup_laplacian(const int n[3], const double h[3], int fd_order, const int bc[3],
                             void* hip_stream, kx_grid** out) {
  const Range range("kx_setup_laplacian");
  if (!n || !h || !bc || !out) return KX_ERR_INVALID_ARG;
  for (int k = 0; k < 3; ++k) {
    if (n[k] < 1 || n[k] > kMaxN) return KX_ERR_INVALID_ARG;
    if (!(std::isfinite(h[k]) && h[k] > 0.0)) return KX_ERR_INVALID_ARG;
    if (bc[k] != KX_BC_DIRICHLET && bc[k] != KX_BC_PERIODIC) return KX_ERR_INVALID_ARG;
  }
  if (!valid_order(fd_order)) return KX_ERR_INVALID_ARG;

  kx_grid* g = new (std::nothrow) kx_grid();
  if (!g) return KX_ERR_OUT_OF_MEMORY;
  {
    static std::atomic<unsigned long long> next_id{1};
    g->id = next_id++;
  }
  for (int k = 0; k < 3; ++k) {
    g->n[k] = n[k];
    g->h[k] = h[k];
    g->bc[k] = bc[k];
  }
  g->order = fd_order;
  g->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&g->device) != hipSuccess) {
    (void)hipGetLastError();
    delete g;
    return KX_ERR_DEVICE;
  }
  Geom& G = g->geom;
  G.n1 = n[0];
  G.n2 = n[1];
  G.n3 = n[2];
  {
    int* me[3] = {&G.me1, &G.me2, &G.me3};
    int* mo[3] = {&G.mo1, &G.mo2, &G.mo3};
    int* pe[3] = {&G.pe1, &G.pe2, &G.pe3};
    int* po[3] = {&G.po1, &G.po2, &G.po3};
    int* pp[3] = {&G.p1, &G.p2, &G.p3};
    for (int k = 0; k < 3; ++k) {
      *mo[k] = n[k] / 2;
      *me[k] = n[k] - n[k] / 2;
      *pe[k] = pad16(*me[k]);
      *po[k] = pad16(*mo[k]);
      *pp[k] = *pe[k] + *po[k];
    }
  }
  G.N = (long long)n[0] * n[1] * n[2];
  G.slab = (long long)G.p1 * G.p2;
  G.slot = G.slab * G.n3;
  G.fsize = G.slab * G.p3;
  {
    int dev = 0, lds = 64 * 1024;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        lds > 0) {
      g->plan_d = make_plan(G, (size_t)lds, sizeof(double));
      g->plan_f = make_plan(G, (size_t)lds, sizeof(float));
      g->plan_s = make_split_plan(G, (size_t)lds);
    } else {
      (void)hipGetLastError();
      g->plan_d = make_plan(G, 64 * 1024, sizeof(double));
      g->plan_f = make_plan(G, 64 * 1024, sizeof(float));
      g->plan_s = make_split_plan(G, 64 * 1024);
    }
  }
  if (const char* env = std::getenv("KX_MAX_SLOTS")) {
    const int v = std::atoi(env);
    if (v >= 1 && v <= 4096) g->max_slots = v;
  }
  g->batch_cap = g->max_slots;

  auto fail = [&](kx_status st) {
    kx_destroy(g);
    return st;
  };
  double* dA = nullptr;
  double* dW = nullptr;
  double* dDiag = nullptr;
  kx_status st = dev_alloc((void**)&dA, sizeof(double) * kMaxN * kMaxN);
  if (st != KX_OK) return fail(st);
  st = dev_alloc((void**)&dW, sizeof(double) * kMaxN * kMaxN);
  if (st != KX_OK) {
    dev_free(dA);
    return fail(st);
  }
  st = dev_alloc((void**)&dDiag, sizeof(double) * 8);
  if (st != KX_OK) {
    dev_free(dA);
    dev_free(dW);
    return fail(st);
  }
  auto cleanup = [&]() {
    dev_free(dA);
    dev_free(dW);
    dev_free(dDiag);
  };
  // Per axis: fold -L_k into its even block E (me x me) and odd block O
  // (mo x mo) in the bases (e_i + e_{n-1-i})/sqrt2, e_m (middle of odd n) and
  // (e_i - e_{n-1-i})/sqrt2; diagonalise both on the device; the stored half
  // eigenvectors are U/sqrt2 except the middle row (kept as is).
  std::vector<double> L, B;
  const double rs = 1.0 / std::sqrt(2.0);
  for (int k = 0; k < 3; ++k) {
    const int nk = n[k], m = nk / 2, me = nk - m, mo = m;
    const int pe = pad16(me), po = pad16(mo);
    if (dev_alloc((void**)&g->dVE[k], sizeof(double) * pe * pe) != KX_OK ||
        dev_alloc((void**)&g->dVET[k], sizeof(double) * pe * pe) != KX_OK ||
        dev_alloc((void**)&g->dLamE[k], sizeof(double) * pe) != KX_OK ||
        dev_alloc((void**)&g->dVO[k], sizeof(double) * std::max(po * po, 1)) != KX_OK ||
        dev_alloc((void**)&g->dVOT[k], sizeof(double) * std::max(po * po, 1)) != KX_OK ||
        dev_alloc((void**)&g->dLamO[k], sizeof(double) * std::max(po, 1)) != KX_OK) {
      cleanup();
      return fail(KX_ERR_OUT_OF_MEMORY);
    }
    L.assign((size_t)nk * nk, 0.0);
    laplacian_1d(nk, h[k], fd_order, bc[k], L.data());
    auto A = [&](int i, int j) { return -L[(size_t)i * nk + j]; };
    std::vector<double> lamE(pe, 0.0), lamO(std::max(po, 1), 0.0);
    std::vector<double> VE((size_t)pe * pe), VO((size_t)std::max(po * po, 1));
    for (int par = 0; par < 2; ++par) {
      const int dim = par == 0 ? me : mo;
      if (dim == 0) continue;
      B.assign((size_t)dim * dim, 0.0);
      for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
          double v;
          if (i < m && j < m) {
            v = par == 0 ? A(i, j) + A(i, nk - 1 - j) : A(i, j) - A(i, nk - 1 - j);
          } else if (i == m && j == m) {
            v = A(m, m);
          } else {
            v = std::sqrt(2.0) * A(i < m ? i : j, m);  // even block only: odd n
          }
          B[(size_t)i * dim + j] = v;
        }
      const int np = par == 0 ? pe : po;
      double* dVh = par == 0 ? g->dVE[k] : g->dVO[k];
      double* dVhT = par == 0 ? g->dVET[k] : g->dVOT[k];
      double* dLam = par == 0 ? g->dLamE[k] : g->dLamO[k];
      const int keep = (par == 0 && (nk & 1)) ? m : -1;
      double diag = 0.0;
      if (hipMemcpyAsync(dA, B.data(), sizeof(double) * dim * dim, hipMemcpyHostToDevice,
                         g->stream) != hipSuccess ||
          launch_jacobi(dA, dW, dim, 60, rs, keep, dLam, dVh, dVhT, np, dDiag, g->stream) !=
              hipSuccess ||
          hipMemcpyAsync(&diag, dDiag, sizeof(double), hipMemcpyDeviceToHost, g->stream) !=
              hipSuccess ||
          hipMemcpyAsync(par == 0 ? lamE.data() : lamO.data(), dLam, sizeof(double) * np,
                         hipMemcpyDeviceToHost, g->stream) != hipSuccess ||
          hipMemcpyAsync(par == 0 ? VE.data() : VO.data(), dVh, sizeof(double) * np * np,
                         hipMemcpyDeviceToHost, g->stream) != hipSuccess ||
          hipStreamSynchronize(g->stream) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return fail(KX_ERR_DEVICE);
      }
      if (diag >= 60.0) {
        cleanup();
        return fail(KX_ERR_NUMERIC);
      }
    }
    // float copies of the half blocks and their transposes
    {
      const int pes = pe * pe, pos = std::max(po * po, 1);
      std::vector<float> fe(pes), fet(pes), fo(pos, 0.0f), fot(pos, 0.0f);
      for (int i = 0; i < pe; ++i)
        for (int a = 0; a < pe; ++a) {
          fe[(size_t)i * pe + a] = (float)VE[(size_t)i * pe + a];
          fet[(size_t)a * pe + i] = (float)VE[(size_t)i * pe + a];
        }
      for (int i = 0; i < po; ++i)
        for (int a = 0; a < po; ++a) {
          fo[(size_t)i * po + a] = (float)VO[(size_t)i * po + a];
          fot[(size_t)a * po + i] = (float)VO[(size_t)i * po + a];
        }
      if (dev_alloc((void**)&g->fVE[k], sizeof(float) * pes) != KX_OK ||
          dev_alloc((void**)&g->fVET[k], sizeof(float) * pes) != KX_OK ||
          dev_alloc((void**)&g->fVO[k], sizeof(float) * pos) != KX_OK ||
          dev_alloc((void**)&g->fVOT[k], sizeof(float) * pos) != KX_OK) {
        cleanup();
        return fail(KX_ERR_OUT_OF_MEMORY);
      }
      if (hipMemcpy(g->fVE[k], fe.data(), sizeof(float) * pes, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(g->fVET[k], fet.data(), sizeof(float) * pes, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(g->fVO[k], fo.data(), sizeof(float) * pos, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(g->fVOT[k], fot.data(), sizeof(float) * pos, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return fail(KX_ERR_DEVICE);
      }
    }
    // three-term bf16 splits of the same blocks
    {
      std::vector<double> vet((size_t)pe * pe), vot((size_t)std::max(po * po, 1), 0.0);
      std::vector<double> ve((size_t)pe * pe), vo((size_t)std::max(po * po, 1), 0.0);
      for (int i = 0; i < pe; ++i)
        for (int a = 0; a < pe; ++a) {
          ve[(size_t)i * pe + a] = VE[(size_t)i * pe + a];
          vet[(size_t)a * pe + i] = VE[(size_t)i * pe + a];
        }
      for (int i = 0; i < po; ++i)
        for (int a = 0; a < po; ++a) {
          vo[(size_t)i * po + a] = VO[(size_t)i * po + a];
          vot[(size_t)a * po + i] = VO[(size_t)i * po + a];
        }
      const std::vector<short> se = split3(ve, pe), set = split3(vet, pe);
      const std::vector<short> so = split3(vo, po), sot = split3(vot, po);
      const std::vector<short> he = split3_f16(ve, pe), het = split3_f16(vet, pe);
      const std::vector<short> ho = split3_f16(vo, po), hot = split3_f16(vot, po);
      short** dst[8] = {&g->sVE[k], &g->sVET[k], &g->sVO[k], &g->sVOT[k],
                        &g->hVE[k], &g->hVET[k], &g->hVO[k], &g->hVOT[k]};
      const std::vector<short>* srcs[8] = {&se, &set, &so, &sot, &he, &het, &ho, &hot};
      for (int b = 0; b < 8; ++b) {
        const size_t bytes = sizeof(short) * srcs[b]->size();
        if (dev_alloc((void**)dst[b], bytes) != KX_OK) {
          cleanup();
          return fail(KX_ERR_OUT_OF_MEMORY);
        }
        if (hipMemcpy(*dst[b], srcs[b]->data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
          (void)hipGetLastError();
          cleanup();
          return fail(KX_ERR_DEVICE);
        }
      }
    }
    // unfold into the full eigensystem (host copy), sorted by eigenvalue
    std::vector<std::pair<double, int>> order;
    for (int a = 0; a < me; ++a) order.push_back({lamE[a], a});
    for (int a = 0; a < mo; ++a) order.push_back({lamO[a], me + a});
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<double, int>& x, const std::pair<double, int>& y) {
                       return x.first < y.first;
                     });
    g->lam_host[k].assign(nk, 0.0);
    g->V_host[k].assign((size_t)nk * nk, 0.0);
    for (int col = 0; col < nk; ++col) {
      const int src = order[col].second;
      g->lam_host[k][col] = order[col].first;
      for (int i = 0; i < me; ++i) {
        double* V = g->V_host[k].data();
        if (src < me) {
          const double v = VE[(size_t)i * pe + src];
          V[(size_t)i * nk + col] = v;
          if (i < m) V[(size_t)(nk - 1 - i) * nk + col] = v;
        } else if (i < m) {
          const double v = VO[(size_t)i * po + (src - me)];
          V[(size_t)i * nk + col] = v;
          V[(size_t)(nk - 1 - i) * nk + col] = -v;
        }
      }
    }
    // orthonormality of the unfolded basis
    double worst = 0.0;
    const double* V = g->V_host[k].data();
    for (int a = 0; a < nk; ++a)
      for (int b = a; b < nk; ++b) {
        double sum = 0.0;
        for (int i = 0; i < nk; ++i) sum += V[(size_t)i * nk + a] * V[(size_t)i * nk + b];
        worst = std::max(worst, std::fabs(sum - (a == b ? 1.0 : 0.0)));
      }
    if (!(worst < 1e-12)) {
      cleanup();
      return fail(KX_ERR_NUMERIC);
    }
  }
  cleanup();
  if (dev_alloc((void**)&g->dEx, sizeof(double) * 2) != KX_OK ||
      dev_alloc((void**)&g->dF, sizeof(double) * (size_t)G.fsize) != KX_OK)
    return fail(KX_ERR_OUT_OF_MEMORY);
  // the no-allocation entry point's scratch array on this device
  st = scratch_init(g->device);
  if (st != KX_OK) return fail(st);
  kx_logf("setup n=(%d, %d, %d) h=(%g, %g, %g) order=%d bc=(%c, %c, %c) device=%d "
          "fwd(slabs %d, kc %d, waves %d) pen(waves %d, lds %zu) inv(slabs %d, kc %d, waves %d)",
          g->n[0], g->n[1], g->n[2], g->h[0], g->h[1], g->h[2], g->order,
          g->bc[0] == KX_BC_PERIODIC ? 'P' : 'D', g->bc[1] == KX_BC_PERIODIC ? 'P' : 'D',
          g->bc[2] == KX_BC_PERIODIC ? 'P' : 'D', g->device, g->plan_d.fwd.slabs, g->plan_d.fwd.kc,
          g->plan_d.fwd.waves, g->plan_d.pen.waves, g->plan_d.pen.lds_bytes, g->plan_d.inv.slabs,
          g->plan_d.inv.kc, g->plan_d.inv.waves);
  *out = g;
  return KX_OK;
}

kx_status kx_destroy(kx_grid* g) {
  if (!g) return KX_OK;
  (void)hipStreamSynchronize(g->stream);
  release_batch_graph(g, true);
  for (int k = 0; k < 3; ++k) {
    dev_free(g->dVE[k]);
    dev_free(g->dVO[k]);
    dev_free(g->dVET[k]);
    dev_free(g->dVOT[k]);
    dev_free(g->dLamE[k]);
    dev_free(g->dLamO[k]);
    dev_free(g->fVE[k]);
    dev_free(g->fVO[k]);
    dev_free(g->fVET[k]);
    dev_free(g->fVOT[k]);
    dev_free(g->sVE[k]);
    dev_free(g->sVO[k]);
    dev_free(g->sVET[k]);
    dev_free(g->sVOT[k]);
    dev_free(g->hVE[k]);
    dev_free(g->hVO[k]);
    dev_free(g->hVET[k]);
    dev_free(g->hVOT[k]);
  }
  free_work(g->ws);
  dev_free(g->dFlag);
  dev_free(g->bl.part);
  dev_free(g->bl.reps);
  dev_free(g->bl.Z);
  dev_free(g->bl.epart);
  dev_free(g->bl.tab);
  dev_free(g->bl.kq);
  dev_free(g->bl.occw);
  dev_free(g->bl.U);
  dev_free(g->bl.W);
  dev_free(g->bl.pairE);
  dev_free(g->dF);
  dev_free(g->dEx);
  dev_free(g->dAcePart);
  dev_free(g->dAceA);
  dev_free(g->dAceLinv);
  dev_free(g->dAceG);
  dev_free(g->dAceU);
  dev_free(g->dAceW);
  dev_free(g->dAceStatus);
  for (hipEvent_t ev : g->prof_ev) (void)hipEventDestroy(ev);
  (void)hipGetLastError();
  delete g;
  return KX_OK;
}

kx_status kx_reserve(kx_grid* g, int norb, int prec, int dtype) {
  if (!g || norb < 0 || norb > 65535) return KX_ERR_INVALID_ARG;
  kx_status st = check_types(g, dtype, prec);
  if (st != KX_OK) return st;
  if ((double)norb * (double)g->geom.N > 4.0e18) return KX_ERR_INVALID_ARG;
  return reserve(g, norb, prec, dtype);
}

kx_status kx_apply_fL(kx_grid* g, int kernel, double omega, int batch, int dtype,
                      const void* rho_dev, void* phi_dev, int prec) {
  if (!g || batch < 0) return KX_ERR_INVALID_ARG;
  if (g->nonorth) return KX_ERR_UNSUPPORTED;  // mixed derivatives couple the real modes
  kx_status st = check_kernel_args(g, kernel, omega);
  if (st != KX_OK) return st;
  st = check_types(g, dtype, prec);
  if (st != KX_OK) return st;
  if (batch == 0) return KX_OK;
  if (!rho_dev || !phi_dev) return KX_ERR_INVALID_ARG;
  if ((double)batch * (double)g->geom.N > 4.0e18) return KX_ERR_INVALID_ARG;
  if (rho_dev == phi_dev) return KX_ERR_INVALID_ARG;
  const Work& w = g->ws;
  if (w.slots < 1 || (prec == KX_PREC_MIXED && !w.T2) || (prec == KX_PREC_FP16X3 && !w.tmax))
    return KX_ERR_STATE;
  // FP16 scales: one per field of a launch, kept in the per-item maxima's
  // companion array sized by the launch
  if (prec == KX_PREC_FP16X3 && w.omax_cap < w.slots) return KX_ERR_STATE;

  if (checks_block_capture(g)) return KX_ERR_STATE;
  const Range range("kx_apply_fL");
  const long long nel = (long long)batch * g->geom.N;
  st = check_finite(g, rho_dev, dtype, nel);
  if (st != KX_OK) return st;
  kx_logf("apply_fL batch=%d prec=%s storage=%s kernel=%d", batch, prec_name(prec),
          dtype == KX_F64 ? "f64" : "f32", kernel);
  hipStream_t s = g->stream;
  g->recording = stream_capturing(s);
  hipError_t e = fill_ftable(g, kernel, omega, s);
  const int chunk = std::min(batch, w.slots);
  const size_t fb = elem_size(dtype) * (size_t)g->geom.N;
  for (int b0 = 0; b0 < batch && e == hipSuccess; b0 += chunk) {
    const int nb = std::min(chunk, batch - b0);
    const void* src = static_cast<const char*>(rho_dev) + fb * b0;
    void* dst = static_cast<char*>(phi_dev) + fb * b0;
    if (prec == KX_PREC_FP16X3)  // the fields' largest magnitudes set the FP16 scales
      e = launch_absmax(src, dtype, (long long)g->geom.N, nb, w.omax, s);
    if (e == hipSuccess)
      e = run_batch(g, w, s, 0, prec, dtype, src, w.fitems, nb, dtype, nullptr, nullptr, dst, 0,
                    0.0);
  }
  g->recording = false;
  KX_HIP(e);
  return check_finite(g, phi_dev, dtype, nel);
}

kx_status kx_apply_fL_multipole(kx_grid* g, int batch, int dtype, const void* rho_dev,
                                void* phi_dev, int prec, int lmax, const double centre[3]) {
  if (!g || batch < 0 || !centre) return KX_ERR_INVALID_ARG;
  if (lmax < 0 || lmax > kMaxMultipoleL) return KX_ERR_INVALID_ARG;
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(centre[k])) return KX_ERR_INVALID_ARG;
  if (!all_dirichlet(g)) return KX_ERR_UNSUPPORTED;
  kx_status st = check_kernel_args(g, KX_KERNEL_COULOMB, 0.0);
  if (st != KX_OK) return st;
  st = check_types(g, dtype, prec);
  if (st != KX_OK) return st;
  if (batch == 0) return KX_OK;
  if (!rho_dev || !phi_dev || rho_dev == phi_dev) return KX_ERR_INVALID_ARG;
  if ((double)batch * (double)g->geom.N > 4.0e18) return KX_ERR_INVALID_ARG;
  const Work& w = g->ws;
  if (w.slots < 1 || !w.mpart || (prec == KX_PREC_MIXED && !w.T2) ||
      (prec == KX_PREC_FP16X3 && (!w.tmax || w.omax_cap < w.slots)))
    return KX_ERR_STATE;

  if (checks_block_capture(g)) return KX_ERR_STATE;
  const Range range("kx_apply_fL_multipole");
  const long long nel = (long long)batch * g->geom.N;
  st = check_finite(g, rho_dev, dtype, nel);
  if (st != KX_OK) return st;
  kx_logf("apply_fL_multipole batch=%d prec=%s lmax=%d centre=(%g, %g, %g)", batch,
          prec_name(prec), lmax, centre[0], centre[1], centre[2]);
  double wfd[13];
  fd_weights_closed_form(g->order, wfd);
  hipStream_t s = g->stream;
  g->recording = stream_capturing(s);
  hipError_t e = fill_ftable(g, KX_KERNEL_COULOMB, 0.0, s);
  const int chunk = std::min(batch, w.slots);
  const size_t fb = elem_size(dtype) * (size_t)g->geom.N;
  for (int b0 = 0; b0 < batch && e == hipSuccess; b0 += chunk) {
    const int nb = std::min(chunk, batch - b0);
    const void* src = static_cast<const char*>(rho_dev) + fb * b0;
    void* dst = static_cast<char*>(phi_dev) + fb * b0;
    // rho + c / (4 pi) into the output fields, then the solve in place
    e = launch_multipole_rhs(dtype, src, dst, nb, g->geom, g->h, centre, wfd, g->order / 2, lmax,
                             w.mpart, w.mmom, s);
    if (e == hipSuccess && prec == KX_PREC_FP16X3)
      e = launch_absmax(dst, dtype, (long long)g->geom.N, nb, w.omax, s);
    if (e == hipSuccess)
      e = run_batch(g, w, s, 0, prec, dtype, dst, w.fitems, nb, dtype, nullptr, nullptr, dst, 0,
                    0.0);
  }
  g->recording = false;
  KX_HIP(e);
  return check_finite(g, phi_dev, dtype, nel);
}

kx_status kx_apply_exchange_multipole(kx_grid* g, int norb, int dtype, const void* psi_dev,
                                      const double* occ_host, void* vxpsi_dev, int prec, int lmax,
                                      const double centre[3]) {
  if (!g || !centre) return KX_ERR_INVALID_ARG;
  if (lmax < 0 || lmax > kMaxMultipoleL) return KX_ERR_INVALID_ARG;
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(centre[k])) return KX_ERR_INVALID_ARG;
  if (!all_dirichlet(g)) return KX_ERR_UNSUPPORTED;
  XPlan xp;
  const Work& w = g->ws;
  kx_status st = plan_exchange(g, w, KX_KERNEL_COULOMB, 0.0, norb, dtype, psi_dev, occ_host,
                               vxpsi_dev, prec, xp);
  if (st != KX_OK) return st;
  if (prec != KX_PREC_FP64) return KX_ERR_UNSUPPORTED;
  hipStream_t s = g->stream;
  if (norb == 0) {
    KX_HIP(launch_zero(g->dEx, sizeof(double), s));
    g->last_norb = 0;
    g->last_pairE = nullptr;
    return KX_OK;
  }
  if (!w.fields || w.dpart_cap < (long long)norb * vx_energy_parts()) return KX_ERR_STATE;
  if (checks_block_capture(g)) return KX_ERR_STATE;
  const Range range("kx_apply_exchange_multipole");
  const long long nel = (long long)norb * g->geom.N;
  st = check_finite(g, psi_dev, dtype, nel);
  if (st != KX_OK) return st;
  kx_logf("apply_exchange_multipole norb=%d lmax=%d centre=(%g, %g, %g) batches=%zu", norb, lmax,
          centre[0], centre[1], centre[2], xp.offsets.size() - 1);
  const Geom& G = g->geom;
  const EigR<double> E = eig_of(g);
  double wfd[13];
  fd_weights_closed_form(g->order, wfd);
  double* T = (double*)w.T;
  g->recording = stream_capturing(s);
  hipError_t e = fill_ftable(g, KX_KERNEL_COULOMB, 0.0, s);
  if (e == hipSuccess) e = launch_put_doubles(xp.occ.data(), norb, w.occ, s);
  if (e == hipSuccess) e = launch_zero(vxpsi_dev, elem_size(dtype) * (size_t)nel, s);
  // rho_ij + c_ij / (4 pi) per pair and the homogeneous solve; with room for
  // a tile's potentials the pairs run in tiles whose potentials one kernel
  // applies to Vx psi (as kx_apply_exchange's two-stage form), else in
  // round-robin batches through the inverse pass's Vx psi epilogue
  auto solve = [&](const Item* it, int nb, bool tile, void* phi) {
    hipError_t r = launch_pair_fields(dtype, psi_dev, it, nb, G.N, w.fields, s);
    if (r == hipSuccess)
      r = launch_multipole_rhs(KX_F64, w.fields, w.fields, nb, G, g->h, centre, wfd,
                               g->order / 2, lmax, w.mpart, w.mmom, s);
    if (r == hipSuccess)
      r = timed(g, s, KX_PHASE_FORWARD, [&] {
        return launch_forward_d(KX_F64, 0, G, g->plan_d.fwd, E, w.fields, w.fitems, nb, T, s);
      });
    if (r == hipSuccess)
      r = timed(g, s, KX_PHASE_PENCIL, [&] {
        return launch_pencil_d(G, g->plan_d.pen, E, g->dF, nb, T, nullptr, s);
      });
    if (r == hipSuccess)
      r = timed(g, s, KX_PHASE_INVERSE, [&] {
        return tile ? launch_inverse_d(KX_F64, 0, G, g->plan_d.inv, E, T, w.fitems, nb, nullptr,
                                       nullptr, phi, s)
                    : launch_inverse_d(dtype, 1, G, g->plan_d.inv, E, T, it, nb, psi_dev, w.occ,
                                       vxpsi_dev, s);
      });
    return r;
  };
  const bool tiles = w.phi && norb <= kXTileMaxOrb &&
                     w.phi_cap >= (long long)kXTile * kXTile * G.N;
  if (tiles) {
    if (e == hipSuccess) e = launch_tile_schedule(norb, w.items, s);
    const int nbk = (norb + kXTile - 1) / kXTile;
    long long off = 0;
    for (int a = 0; a < nbk && e == hipSuccess; ++a)
      for (int b = a; b < nbk && e == hipSuccess; ++b) {
        const int npt = xtile_pairs(a, b, norb);
        for (int p0 = 0; p0 < npt && e == hipSuccess; p0 += w.slots)
          e = solve(w.items + off + p0, std::min(w.slots, npt - p0), true,
                    w.phi + (long long)p0 * G.N);
        off += npt;
        if (e == hipSuccess)
          e = timed(g, s, KX_PHASE_ACCUM, [&] {
            return launch_tile_accumulate(dtype, KX_F64, w.phi, a, b, norb, G.N, psi_dev, w.occ,
                                          vxpsi_dev, s);
          });
      }
  } else {
    if (e == hipSuccess) e = launch_schedule(norb, w.items, s);
    for (size_t b = 0; e == hipSuccess && b + 1 < xp.offsets.size(); ++b) {
      const int o0 = xp.offsets[b], nb = xp.offsets[b + 1] - o0;
      if (nb > 0) e = solve(w.items + o0, nb, false, nullptr);
    }
  }
  // E_x = 1/4 sum_j occ_j <psi_j, (Vx psi)_j>_h (the boundary values make the
  // pair solve non-symmetric, so the energy is taken from the operator)
  if (e == hipSuccess)
    e = launch_vx_energy(dtype, psi_dev, vxpsi_dev, norb, G.N, w.occ,
                         g->h[0] * g->h[1] * g->h[2], w.dpart, g->dEx, s);
  g->recording = false;
  KX_HIP(e);
  g->last_norb = 0;  // no per-pair energies on this path
  g->last_pairE = nullptr;
  st = check_finite(g, vxpsi_dev, dtype, nel);
  return st != KX_OK ? st : check_finite(g, g->dEx, KX_F64, 1);
}

kx_status kx_apply_exchange(kx_grid* g, int kernel, double omega, int norb, int dtype,
                            const void* psi_dev, const double* occ_host, void* vxpsi_dev,
                            int prec) {
  if (!g) return KX_ERR_INVALID_ARG;
  XPlan xp;
  kx_status st = plan_exchange(g, g->ws, kernel, omega, norb, dtype, psi_dev, occ_host, vxpsi_dev,
                               prec, xp);
  if (st != KX_OK) return st;
  if (checks_block_capture(g)) return KX_ERR_STATE;
  const Range range("kx_apply_exchange");
  const long long nel = (long long)norb * g->geom.N;
  st = check_finite(g, psi_dev, dtype, nel);
  if (st != KX_OK) return st;
  kx_logf("apply_exchange norb=%d prec=%s storage=%s kernel=%d batches=%zu", norb,
          prec_name(prec), dtype == KX_F64 ? "f64" : "f32", kernel,
          xp.offsets.empty() ? (size_t)0 : xp.offsets.size() - 1);
  g->recording = stream_capturing(g->stream);
  const hipError_t e = enqueue_exchange(g, xp, g->ws, g->stream);
  g->recording = false;
  KX_HIP(e);
  g->last_norb = norb;
  g->last_pairE = g->ws.pairE;
  st = check_finite(g, vxpsi_dev, dtype, nel);
  return st != KX_OK ? st : check_finite(g, g->dEx, KX_F64, norb > 0 ? 1 : 0);
}

kx_status kx_apply_exchange_noalloc(kx_grid* g, int kernel, double omega, int norb, int dtype,
                                    const void* psi_dev, const double* occ_host, void* vxpsi_dev,
                                    int prec) {
  if (!g || norb < 0 || norb > 65535) return KX_ERR_INVALID_ARG;
  if (prec < KX_PREC_FP64 || prec > KX_PREC_MIXED) return KX_ERR_INVALID_ARG;
  Work w;
  kx_status st = carve_scratch(g, norb, prec, w);
  if (st != KX_OK) return st;
  XPlan xp;
  st = plan_exchange(g, w, kernel, omega, norb, dtype, psi_dev, occ_host, vxpsi_dev, prec, xp);
  if (st != KX_OK) return st;
  if (checks_block_capture(g)) return KX_ERR_STATE;
  const Range range("kx_apply_exchange_noalloc");
  const long long nel = (long long)norb * g->geom.N;
  st = check_finite(g, psi_dev, dtype, nel);
  if (st != KX_OK) return st;
  kx_logf("apply_exchange_noalloc norb=%d prec=%s launch slots=%d", norb, prec_name(prec), w.slots);
  hipStream_t s = g->stream;
  // earlier calls on this device left other shapes in the shared array: the
  // intermediates' padded rows must read as zero
  hipError_t e = hipSuccess;
  if (norb > 0) {
    e = launch_zero(w.T, w.tbytes * w.slots, s);
    if (e == hipSuccess && w.T2) e = launch_zero(w.T2, sizeof(float) * g->geom.slot * w.slots, s);
  }
  g->capturing = true;  // no timing events: nothing is created on this path
  if (e == hipSuccess) e = enqueue_exchange(g, xp, w, s);
  g->capturing = false;
  KX_HIP(e);
  g->last_norb = norb;
  g->last_pairE = w.pairE;
  st = check_finite(g, vxpsi_dev, dtype, nel);
  return st != KX_OK ? st : check_finite(g, g->dEx, KX_F64, norb > 0 ? 1 : 0);
}

kx_status kx_set_cell(kx_grid* g, const double lattice[9]) {
  if (!g) return KX_ERR_INVALID_ARG;
  double gm[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  double jac = 1.0;
  bool nonorth = false;
  if (lattice) {
    // E: the unit lattice directions as columns
    double E[3][3];
    for (int a = 0; a < 3; ++a) {
      double nrm = 0.0;
      for (int i = 0; i < 3; ++i) {
        if (!std::isfinite(lattice[3 * a + i])) return KX_ERR_INVALID_ARG;
        nrm += lattice[3 * a + i] * lattice[3 * a + i];
      }
      nrm = std::sqrt(nrm);
      if (!(nrm > 0.0) || !std::isfinite(nrm)) return KX_ERR_INVALID_ARG;
      for (int i = 0; i < 3; ++i) E[i][a] = lattice[3 * a + i] / nrm;
    }
    const double det = E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
                       E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
                       E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
    if (!(std::fabs(det) > 1e-6)) return KX_ERR_INVALID_ARG;  // (nearly) flat cell
    // E^-1 by the adjugate, then g = E^-1 E^-T
    double Ei[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        const int r1 = (c + 1) % 3, r2 = (c + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
        Ei[r][c] = (E[r1][c1] * E[r2][c2] - E[r1][c2] * E[r2][c1]) / det;
      }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double v = 0.0;
        for (int i = 0; i < 3; ++i) v += Ei[a][i] * Ei[b][i];
        gm[a][b] = v;
      }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        if (a != b && std::fabs(gm[a][b]) > 1e-14) nonorth = true;
    if (nonorth) {
      if (!all_periodic(g)) return KX_ERR_UNSUPPORTED;
      jac = std::fabs(det);
    } else {  // orthonormal directions: the orthogonal cell
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) gm[a][b] = a == b ? 1.0 : 0.0;
    }
  }
  g->nonorth = nonorth;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) g->cell_g[a][b] = gm[a][b];
  g->cell_jac = jac;
  g->zero.tol = zero_tolerance(g);
  ++g->gen;  // recorded work carries the metric in its kernel arguments
  kx_logf("cell %s g=[%g %g %g; %g %g %g; %g %g %g] |det E|=%g",
          nonorth ? "non-orthogonal" : "orthogonal", gm[0][0], gm[0][1], gm[0][2], gm[1][0],
          gm[1][1], gm[1][2], gm[2][0], gm[2][1], gm[2][2], jac);
  return KX_OK;
}

kx_status kx_set_zero_mode(kx_grid* g, int enable, double value) {
  if (!g || (enable && !std::isfinite(value))) return KX_ERR_INVALID_ARG;
  g->zero.on = enable ? 1 : 0;
  g->zero.val = enable ? value : 0.0;
  g->zero.tol = zero_tolerance(g);
  ++g->gen;  // recorded work carries the value in its kernel arguments
  kx_logf("zero mode %s value %g tolerance %g", enable ? "on" : "off", value, g->zero.tol);
  return KX_OK;
}

kx_status kx_set_checks(kx_grid* g, int flags) {
  if (!g || (flags & ~KX_CHECK_FINITE)) return KX_ERR_INVALID_ARG;
  if ((flags & KX_CHECK_FINITE) && !g->dFlag) {
    const kx_status st = dev_alloc((void**)&g->dFlag, sizeof(unsigned));
    if (st != KX_OK) return st;
  }
  g->checks = flags;
  kx_logf("checks 0x%x", flags);
  return KX_OK;
}

kx_status kx_reserve_bloch(kx_grid* g, int nk, int norb) {
  if (!g || nk < 0 || nk > kMaxKpoints || norb < 0 || (nk == 0 && norb != 0))
    return KX_ERR_INVALID_ARG;
  const long long M = (long long)nk * norb;
  if (M > 65535 || (double)M * (double)g->geom.N > 1.0e18) return KX_ERR_INVALID_ARG;
  kx_status st = bloch_map(g);
  if (st != KX_OK) return st;
  st = reserve_slots(g, g->max_slots, false, false);
  if (st != KX_OK) return st;
  auto& B = g->bl;
  const Geom& G = g->geom;
  const int nb = bloch_batch(g);
  if (nb < 1) return KX_ERR_STATE;
  const int K = std::max(nk, 2);
  st = grow(g, &B.Z, &B.z_cap, 2LL * nb * bloch_field_stride(G));
  if (st == KX_OK)
    st = grow(g, &B.epart, &B.epart_cap, (long long)nb * bloch_couple_waves(bloch_reps(g)));
  if (st == KX_OK) st = grow(g, &B.tab, &B.tab_cap, (long long)K * K * 3 * kBlochTab * B.pmax);
  if (st == KX_OK) st = grow(g, &B.kq, &B.kq_cap, 3LL * K);
  if (st == KX_OK && M > 0) st = grow(g, &B.occw, &B.occw_cap, M);
  if (st == KX_OK && M > 0) st = grow(g, &B.U, &B.u_cap, 2 * M * G.N);
  if (st == KX_OK && M > 0) st = grow(g, &B.W, &B.w_cap, 2 * M * G.N);
  if (st == KX_OK && M > 0) st = grow(g, &B.pairE, &B.pairE_cap, M * (M + 1) / 2);
  return st;
}

kx_status kx_apply_fL_bloch(kx_grid* g, int kernel, double omega, int batch, const double theta[3],
                            const void* rho_dev, void* phi_dev, int prec) {
  if (!g || batch < 0 || !theta) return KX_ERR_INVALID_ARG;
  if (kernel != KX_KERNEL_COULOMB && kernel != KX_KERNEL_ERFC) return KX_ERR_INVALID_ARG;
  if (kernel == KX_KERNEL_ERFC && !(std::isfinite(omega) && omega > 0.0)) return KX_ERR_INVALID_ARG;
  if (prec < KX_PREC_FP64 || prec > KX_PREC_MIXED) return KX_ERR_INVALID_ARG;
  BlochT th;
  bool zero_mode = true;  // the spectrum of -L(theta) contains 0
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(theta[a])) return KX_ERR_INVALID_ARG;
    th.t[a] = theta[a] / (2.0 * M_PI);
    if (g->bc[a] != KX_BC_PERIODIC) {
      if (theta[a] != 0.0) return KX_ERR_INVALID_ARG;
      zero_mode = false;
    } else if (th.t[a] != std::rint(th.t[a])) {
      zero_mode = false;
    }
  }
  if (kernel == KX_KERNEL_COULOMB && zero_mode && !g->zero.on) return KX_ERR_SINGULAR;
  if (prec != KX_PREC_FP64) return KX_ERR_UNSUPPORTED;
  if (batch == 0) return KX_OK;
  if (!rho_dev || !phi_dev || rho_dev == phi_dev) return KX_ERR_INVALID_ARG;
  if ((double)batch * (double)g->geom.N > 1.0e18) return KX_ERR_INVALID_ARG;
  if (!bloch_reserved(g, 0, 0)) return KX_ERR_STATE;
  if (checks_block_capture(g)) return KX_ERR_STATE;
  const Range range("kx_apply_fL_bloch");
  const long long nel = 2LL * batch * g->geom.N;
  kx_status st = check_finite(g, rho_dev, KX_F64, nel);
  if (st != KX_OK) return st;
  kx_logf("apply_fL_bloch batch=%d theta=(%g, %g, %g) kernel=%d%s", batch, theta[0], theta[1],
          theta[2], kernel, g->nonorth ? " non-orthogonal cell" : "");

  const Geom& G = g->geom;
  hipStream_t s = g->stream;
  g->recording = stream_capturing(s);
  // class 1 of a two-point table: theta = 2 pi (kq[0] - kq[1]) with kq[1] = 0
  const double kq[6] = {th.t[0], th.t[1], th.t[2], 0.0, 0.0, 0.0};
  hipError_t e = launch_put_doubles(kq, 6, g->bl.kq, s);
  if (e == hipSuccess)
    e = launch_bloch_table(bloch_axes(g), g->bl.kq, 2, g->bl.pmax, g->bl.tab, s);
  const int chunk = bloch_batch(g);
  const size_t fb = 2 * sizeof(double) * (size_t)G.N;
  const PairMap pm{0, 0, 0, 1, 2, 1};
  for (int b0 = 0; b0 < batch && e == hipSuccess; b0 += chunk) {
    const int nb = std::min(chunk, batch - b0);
    const double* src = (const double*)((const char*)rho_dev + fb * b0);
    double* dst = (double*)((char*)phi_dev + fb * b0);
    e = launch_bloch_fields(0, G, th, nb, src, g->bl.Z, s);
    if (e == hipSuccess) e = bloch_solve(g, kernel, omega, pm, nb, s);
    if (e == hipSuccess) e = launch_bloch_fields(1, G, th, nb, g->bl.Z, dst, s);
  }
  g->recording = false;
  KX_HIP(e);
  return check_finite(g, phi_dev, KX_F64, nel);
}

kx_status kx_apply_exchange_bloch(kx_grid* g, int kernel, double omega, int nk, int norb,
                                  const double* kpts_host, const double* wk_host,
                                  const double* occ_host, const void* psi_dev, void* vxpsi_dev,
                                  int prec) {
  if (!g || nk < 1 || nk > kMaxKpoints || norb < 0) return KX_ERR_INVALID_ARG;
  kx_status st = check_kernel_args(g, kernel, omega);
  if (st != KX_OK) return st;
  if (prec < KX_PREC_FP64 || prec > KX_PREC_MIXED) return KX_ERR_INVALID_ARG;
  if (!kpts_host || !wk_host || (norb > 0 && !occ_host)) return KX_ERR_INVALID_ARG;
  const long long M = (long long)nk * norb;
  if (M > 65535) return KX_ERR_INVALID_ARG;
  std::vector<double> kq(3 * (size_t)std::max(nk, 2), 0.0), occw((size_t)M);
  for (int k = 0; k < nk; ++k) {
    if (!std::isfinite(wk_host[k])) return KX_ERR_INVALID_ARG;
    for (int a = 0; a < 3; ++a) {
      const double v = kpts_host[3 * k + a];
      if (!std::isfinite(v)) return KX_ERR_INVALID_ARG;
      if (g->bc[a] != KX_BC_PERIODIC && v != 0.0) return KX_ERR_INVALID_ARG;
      kq[3 * (size_t)k + a] = v;
    }
    for (int n = 0; n < norb; ++n) {
      const double o = occ_host[(size_t)k * norb + n];
      if (!std::isfinite(o)) return KX_ERR_INVALID_ARG;
      occw[(size_t)k * norb + n] = wk_host[k] * o;
    }
  }
  if (prec != KX_PREC_FP64) return KX_ERR_UNSUPPORTED;
  hipStream_t s = g->stream;
  if (M == 0) {
    KX_HIP(launch_zero(g->dEx, sizeof(double), s));
    g->last_norb = 0;
    g->last_pairE = nullptr;
    return KX_OK;
  }
  if (!psi_dev || !vxpsi_dev || psi_dev == vxpsi_dev) return KX_ERR_INVALID_ARG;
  if (!bloch_reserved(g, nk, norb)) return KX_ERR_STATE;
  if (checks_block_capture(g)) return KX_ERR_STATE;
  const Range range("kx_apply_exchange_bloch");
  const long long nel = 2 * M * g->geom.N;
  st = check_finite(g, psi_dev, KX_F64, nel);
  if (st != KX_OK) return st;
  kx_logf("apply_exchange_bloch nk=%d norb=%d state pairs=%lld kernel=%d%s", nk, norb,
          M * (M + 1) / 2, kernel, g->nonorth ? " non-orthogonal cell" : "");

  const Geom& G = g->geom;
  auto& B = g->bl;
  g->recording = stream_capturing(s);
  hipError_t e = launch_put_doubles(kq.data(), 3 * nk, B.kq, s);
  if (e == hipSuccess) e = launch_put_doubles(occw.data(), (int)M, B.occw, s);
  if (e == hipSuccess) e = launch_bloch_table(bloch_axes(g), B.kq, nk, B.pmax, B.tab, s);
  if (e == hipSuccess)
    e = launch_bloch_orbitals(0, G, (int)M, norb, B.kq, (const double*)psi_dev, B.U, B.W, s);
  const int nblk = bloch_couple_waves(bloch_reps(g));
  const double dV = cell_dV(g);
  // one launch per tile of kTileR x kTileC state pairs of the upper triangle,
  // column blocks outer, row blocks inner
  for (int c0 = 0; c0 < (int)M && e == hipSuccess; c0 += kTileC)
    for (int r0 = 0; r0 < std::min((int)M, c0 + kTileC) && e == hipSuccess; r0 += kTileR) {
      const int nb = tile_pairs(r0, c0, (int)M);
      if (nb == 0) continue;
      const PairMap pm{r0, c0, (int)M, norb, nk, 0};
      e = launch_bloch_products(G, B.U, pm, nb, B.Z, s);
      if (e == hipSuccess) e = bloch_solve(g, kernel, omega, pm, nb, s);
      if (e == hipSuccess)
        e = timed(g, s, KX_PHASE_ENERGY, [&] {
          return launch_bloch_pair_sums(B.epart, nblk, nb, pm, dV, B.pairE, s);
        });
      if (e == hipSuccess) e = launch_bloch_update(G, B.U, B.Z, pm, nb, B.occw, B.W, s);
    }
  if (e == hipSuccess)
    e = launch_bloch_orbitals(1, G, (int)M, norb, B.kq, nullptr, (double*)vxpsi_dev, B.W, s);
  if (e == hipSuccess) e = launch_bloch_energy(B.pairE, (int)M, B.occw, g->dEx, s);
  g->recording = false;
  KX_HIP(e);
  g->last_norb = 0;  // kx_pair_energies covers real orbitals only
  g->last_pairE = nullptr;
  st = check_finite(g, vxpsi_dev, KX_F64, nel);
  return st != KX_OK ? st : check_finite(g, g->dEx, KX_F64, 1);
}

kx_status kx_batch_apply_exchange(int nsys, kx_grid* const* grids, const int* kernels,
                                  const double* omegas, const int* norbs, int dtype,
                                  const void* const* psi_dev, const double* const* occ_host,
                                  void* const* vxpsi_dev, int prec, double* ex_out) {
  const Range range("kx_batch_apply_exchange");
  if (nsys < 1 || nsys > 256 || !grids || !kernels || !omegas || !norbs || !psi_dev || !occ_host ||
      !vxpsi_dev)
    return KX_ERR_INVALID_ARG;
  for (int k = 0; k < nsys; ++k) {
    if (!grids[k]) return KX_ERR_INVALID_ARG;
    for (int m = 0; m < k; ++m)
      if (grids[m] == grids[k]) return KX_ERR_INVALID_ARG;  // one workspace per system
  }
  std::vector<XPlan> xps(nsys);
  for (int k = 0; k < nsys; ++k) {  // validation first, then the workspaces
    kx_status st = check_types(grids[k], dtype, prec);
    if (st != KX_OK) return st;
    if (norbs[k] < 0 || norbs[k] > 65535) return KX_ERR_INVALID_ARG;
    Work none;
    st = plan_exchange(grids[k], none, kernels[k], omegas[k], 0, dtype, psi_dev[k], occ_host[k],
                       vxpsi_dev[k], prec, xps[k]);
    if (st != KX_OK) return st;
  }
  for (int k = 0; k < nsys; ++k) {
    kx_status st = reserve(grids[k], norbs[k], prec, dtype);
    if (st == KX_OK)
      st = plan_exchange(grids[k], grids[k]->ws, kernels[k], omegas[k], norbs[k], dtype,
                         psi_dev[k], occ_host[k], vxpsi_dev[k], prec, xps[k]);
    if (st != KX_OK) return st;
  }
  // any earlier work on the systems' own streams comes first
  for (int k = 0; k < nsys; ++k) KX_HIP(hipStreamSynchronize(grids[k]->stream));

  kx_grid* o = grids[0];
  auto& b = o->batch;
  std::vector<unsigned long long> key;
  for (int k = 0; k < nsys; ++k) {
    unsigned long long om;
    std::memcpy(&om, &omegas[k], sizeof om);
    key.insert(key.end(), {grids[k]->id, grids[k]->gen, (unsigned long long)kernels[k], om,
                           (unsigned long long)norbs[k], (unsigned long long)prec,
                           (unsigned long long)dtype, (unsigned long long)(uintptr_t)psi_dev[k],
                           (unsigned long long)(uintptr_t)vxpsi_dev[k],
                           (unsigned long long)grids[k]->batch_cap});
    // the occupations travel as kernel arguments of the recorded work
    for (int i = 0; i < norbs[k]; ++i) {
      unsigned long long o;
      std::memcpy(&o, &occ_host[k][i], sizeof o);
      key.push_back(o);
    }
  }
  if (!(b.exec && b.key == key)) {
    release_batch_graph(o, false);
    if (!b.origin) KX_HIP(hipStreamCreateWithFlags(&b.origin, hipStreamNonBlocking));
    if (!b.fork) KX_HIP(hipEventCreateWithFlags(&b.fork, hipEventDisableTiming));
    while ((int)b.branch.size() < nsys) {
      hipStream_t s;
      KX_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      b.branch.push_back(s);
      hipEvent_t e;
      KX_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      b.join.push_back(e);
    }
    // record: fork from the origin stream, one branch per system, join back
    KX_HIP(hipStreamBeginCapture(b.origin, hipStreamCaptureModeRelaxed));
    hipError_t e = hipEventRecord(b.fork, b.origin);
    for (int k = 0; k < nsys && e == hipSuccess; ++k) {
      e = hipStreamWaitEvent(b.branch[k], b.fork, 0);
      if (e != hipSuccess) break;
      grids[k]->capturing = true;
      e = enqueue_exchange(grids[k], xps[k], grids[k]->ws, b.branch[k]);
      grids[k]->capturing = false;
      if (e != hipSuccess) break;
      e = hipEventRecord(b.join[k], b.branch[k]);
      if (e == hipSuccess) e = hipStreamWaitEvent(b.origin, b.join[k], 0);
    }
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b.origin, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      return KX_ERR_DEVICE;
    }
    b.graph = graph;
    if (hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGetLastError();
      release_batch_graph(o, false);
      return KX_ERR_DEVICE;
    }
    b.key = key;
  }
  KX_HIP(hipGraphLaunch(b.exec, b.origin));
  KX_HIP(hipStreamSynchronize(b.origin));
  for (int k = 0; k < nsys; ++k) {
    grids[k]->last_norb = norbs[k];
    grids[k]->last_pairE = grids[k]->ws.pairE;
    if (ex_out)
      KX_HIP(hipMemcpy(&ex_out[k], grids[k]->dEx, sizeof(double), hipMemcpyDeviceToHost));
  }
  return KX_OK;
}

kx_status kx_autotune(kx_grid* g, int prec, int dtype, int items, int verify,
                      const char* cache_path) {
  const Range range("kx_autotune");
  if (!g || dtype < KX_F64 || dtype > KX_F32) return KX_ERR_INVALID_ARG;
  if (prec == KX_PREC_MIXED) {  // its forward and pencil passes are FP64's, its inverse BF16X3's
    const kx_status st = kx_autotune(g, KX_PREC_FP64, dtype, items, verify, cache_path);
    return st != KX_OK ? st : kx_autotune(g, KX_PREC_BF16X3, dtype, items, verify, cache_path);
  }
  if (prec == KX_PREC_FP16X3) prec = KX_PREC_BF16X3;  // the same split kernels' shapes
  if (prec != KX_PREC_FP64 && prec != KX_PREC_FP32 && prec != KX_PREC_BF16X3)
    return KX_ERR_INVALID_ARG;
  const Geom& G = g->geom;
  // the storage the transform kernels see (reduced precision on FP64 storage
  // runs on FP32 working copies)
  const int dtype_w = (prec != KX_PREC_FP64 && dtype == KX_F64) ? KX_F32 : dtype;
  const int kind = prec == KX_PREC_FP64 ? 0 : (prec == KX_PREC_FP32 ? 1 : 2);
  Plan& plan = kind == 0 ? g->plan_d : (kind == 1 ? g->plan_f : g->plan_s);
  int dev = 0, lds = 64 * 1024;
  hipDeviceProp_t prop;
  KX_HIP(hipGetDevice(&dev));
  KX_HIP(hipGetDeviceProperties(&prop, dev));
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
    (void)hipGetLastError();
    lds = 64 * 1024;
  }
  char key[256];
  std::snprintf(key, sizeof key, "kx-tune-v2 %d %d %d %d %d %d %d %d %s %d", G.n1, G.n2, G.n3,
                g->bc[0], g->bc[1], g->bc[2], kind, dtype_w, prop.gcnArchName,
                prop.multiProcessorCount);
  // cached result: "<key> | fwd qsplit slabs waves kc vlds lds | pen waves lds per | inv slabs waves kc vlds lds"
  if (cache_path && !verify) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char line[512];
      bool found = false;
      while (std::fgets(line, sizeof line, f)) {
        const size_t kl = std::strlen(key);
        if (std::strncmp(line, key, kl) != 0 || line[kl] != ' ') continue;
        SlabPlan fw, iv;
        PencilPlan pn;
        int fv = 0, ivv = 0;
        unsigned long long fl = 0, pl = 0, il = 0;
        if (std::sscanf(line + kl, " | fwd %d %d %d %d %d %llu | pen %d %llu %d | inv %d %d %d %d %llu",
                        &fw.qsplit, &fw.slabs, &fw.waves, &fw.kc, &fv, &fl, &pn.waves, &pl,
                        &pn.per, &iv.slabs, &iv.waves, &iv.kc, &ivv, &il) == 14) {
          fw.vlds = fv != 0;
          fw.lds_bytes = fl;
          pn.lds_bytes = pl;
          iv.vlds = ivv != 0;
          iv.lds_bytes = il;
          // accept only a shape the planner itself proposes
          std::vector<SlabPlan> cf, ci;
          std::vector<PencilPlan> cp;
          plan_candidates(G, (size_t)lds, kind, cf, cp, ci, elem_size(dtype_w));
          auto same = [](const SlabPlan& a, const SlabPlan& b) {
            return a.qsplit == b.qsplit && a.slabs == b.slabs && a.waves == b.waves &&
                   a.kc == b.kc && a.vlds == b.vlds && a.lds_bytes == b.lds_bytes;
          };
          bool okf = false, okp = false, oki = false;
          for (auto& c : cf) okf = okf || same(c, fw);
          for (auto& c : ci) oki = oki || same(c, iv);
          for (auto& c : cp)
            okp = okp || (c.waves == pn.waves && c.lds_bytes == pn.lds_bytes && c.per == pn.per);
          if (okf && okp && oki) {
            plan.fwd = fw;
            plan.pen = pn;
            plan.inv = iv;
            ++g->gen;
            found = true;
          }
        }
      }
      std::fclose(f);
      if (found) return KX_OK;
    }
  }

  const int nb = std::max(1, std::min(items > 0 ? items : g->max_slots, g->max_slots));
  const int norb_t = 2 * nb;
  const size_t esw = elem_size(dtype_w);
  const size_t fbytes = esw * (size_t)norb_t * G.N;
  const size_t tbytes = (kind == 0 ? sizeof(double) : sizeof(float)) * (size_t)nb * G.slot;
  kx_status st = reserve_slots(g, nb, false, false);
  if (st != KX_OK) return st;
  KX_HIP(fill_ftable(g, KX_KERNEL_ERFC, 0.106, g->stream));
  std::vector<Item> its(nb);
  for (int k = 0; k < nb; ++k) its[k] = {2 * k, 2 * k + 1};
  void *psi = nullptr, *vx = nullptr, *tsave = nullptr, *ref = nullptr;
  double* occ = nullptr;
  Item* dit = nullptr;
  unsigned long long* cnt = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto release = [&]() {
    (void)hipStreamSynchronize(g->stream);
    dev_free(psi);
    dev_free(vx);
    dev_free(tsave);
    dev_free(ref);
    dev_free(occ);
    dev_free(dit);
    dev_free(cnt);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (dev_alloc(&psi, fbytes) != KX_OK || dev_alloc(&vx, fbytes) != KX_OK ||
      dev_alloc(&tsave, tbytes) != KX_OK || dev_alloc(&ref, std::max(tbytes, fbytes)) != KX_OK ||
      dev_alloc((void**)&occ, sizeof(double) * norb_t) != KX_OK ||
      dev_alloc((void**)&dit, sizeof(Item) * nb) != KX_OK ||
      dev_alloc((void**)&cnt, sizeof(unsigned long long)) != KX_OK) {
    release();
    return KX_ERR_OUT_OF_MEMORY;
  }
  if (hipMemcpy(dit, its.data(), sizeof(Item) * nb, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    release();
    return KX_ERR_DEVICE;
  }
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    release();
    return KX_ERR_DEVICE;
  }
  hipStream_t s = g->stream;
  const std::vector<double> ones(norb_t, 1.0);
  hipError_t he = hipMemcpy(occ, ones.data(), sizeof(double) * norb_t, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = launch_pattern(psi, (long long)norb_t * G.N, dtype_w == KX_F64, s);
  if (he != hipSuccess) {
    (void)hipGetLastError();
    release();
    return KX_ERR_DEVICE;
  }
  auto fwd = [&](const SlabPlan& p) -> hipError_t {
    if (kind == 0)
      return launch_forward_d(dtype_w, 1, G, p, eig_of(g), psi, dit, nb, (double*)g->ws.T, s);
    if (kind == 1)
      return launch_forward_f(dtype_w, 1, G, p, eigf_of(g), psi, dit, nb, (float*)g->ws.T, s);
    return launch_forward_s(dtype_w, 1, G, p, eigs_of(g), psi, dit, nb, (float*)g->ws.T, s);
  };
  auto pen = [&](const PencilPlan& p) -> hipError_t {
    if (kind == 0)
      return launch_pencil_d(G, p, eig_of(g), g->dF, nb, (double*)g->ws.T, g->ws.epart, s);
    if (kind == 1)
      return launch_pencil_f(G, p, eigf_of(g), g->dF, nb, (float*)g->ws.T, g->ws.epart, s);
    return launch_pencil_s(G, p, eigs_of(g), g->dF, nb, (float*)g->ws.T, g->ws.epart, s);
  };
  auto inv = [&](const SlabPlan& p) -> hipError_t {
    if (kind == 0)
      return launch_inverse_d(dtype_w, 1, G, p, eig_of(g), (const double*)g->ws.T, dit, nb, psi, occ,
                              vx, s);
    if (kind == 1)
      return launch_inverse_f(dtype_w, 1, G, p, eigf_of(g), (const float*)g->ws.T, dit, nb, psi,
                              occ, vx, s);
    return launch_inverse_s(dtype_w, 1, G, p, eigs_of(g), (const float*)g->ws.T, dit, nb, psi, occ,
                            vx, s);
  };
  // mean time of three launches after one warm-up
  // best of three rounds of three launches (shapes within a few per cent of
  // each other are otherwise ranked by noise)
  auto timeit = [&](auto&& launch, auto&& reset, float& ms) -> hipError_t {
    hipError_t e = reset();
    if (e == hipSuccess) e = launch();
    ms = 1e30f;
    for (int round = 0; round < 3 && e == hipSuccess; ++round) {
      float t = 0.f;
      e = reset();
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch();
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
      ms = std::min(ms, t / 3.0f);
    }
    return e;
  };
  // bitwise agreement of buf with the reference copy
  auto same_as_ref = [&](const void* buf, size_t bytes, bool& same) -> hipError_t {
    unsigned long long c = 0;
    hipError_t e = hipMemsetAsync(cnt, 0, sizeof c, s);
    if (e == hipSuccess) e = launch_diff(buf, ref, bytes, cnt, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&c, cnt, sizeof c, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    same = c == 0;
    return e;
  };
  auto none = [&]() -> hipError_t { return hipSuccess; };
  auto fail_dev = [&]() {
    (void)hipGetLastError();
    release();
    return KX_ERR_DEVICE;
  };

  std::vector<SlabPlan> cf, ci;
  std::vector<PencilPlan> cp;
  plan_candidates(G, (size_t)lds, kind, cf, cp, ci, elem_size(dtype_w));
  if (cf.empty() || cp.empty() || ci.empty()) {
    release();
    return KX_ERR_UNSUPPORTED;
  }
  bool all_same = true;
  // forward: reference with the current shape, then every candidate
  if (fwd(plan.fwd) != hipSuccess ||
      hipMemcpyAsync(ref, g->ws.T, tbytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return fail_dev();
  float best = 1e30f;
  SlabPlan bf = plan.fwd;
  for (const SlabPlan& c : cf) {
    float ms = 0;
    if (timeit([&] { return fwd(c); }, none, ms) != hipSuccess) return fail_dev();
    if (verify) {
      bool same = false;
      if (same_as_ref(g->ws.T, tbytes, same) != hipSuccess) return fail_dev();
      all_same = all_same && same;
    }
    if (ms < best) {
      best = ms;
      bf = c;
    }
  }
  // pencil: each run starts from the forward output
  if (fwd(bf) != hipSuccess ||
      hipMemcpyAsync(tsave, g->ws.T, tbytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      pen(plan.pen) != hipSuccess ||
      hipMemcpyAsync(ref, g->ws.T, tbytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return fail_dev();
  auto restore_t = [&]() { return hipMemcpyAsync(g->ws.T, tsave, tbytes, hipMemcpyDeviceToDevice, s); };
  best = 1e30f;
  PencilPlan bp = plan.pen;
  for (const PencilPlan& c : cp) {
    float ms = 0;
    if (timeit([&] { return pen(c); }, restore_t, ms) != hipSuccess) return fail_dev();
    if (verify) {
      bool same = false;
      if (restore_t() != hipSuccess || pen(c) != hipSuccess ||
          same_as_ref(g->ws.T, tbytes, same) != hipSuccess)
        return fail_dev();
      all_same = all_same && same;
    }
    if (ms < best) {
      best = ms;
      bp = c;
    }
  }
  // inverse: from the pencil output, into a cleared Vx psi
  if (restore_t() != hipSuccess || pen(bp) != hipSuccess) return fail_dev();
  auto clear_vx = [&]() { return launch_zero(vx, fbytes, s); };
  if (clear_vx() != hipSuccess || inv(plan.inv) != hipSuccess ||
      hipMemcpyAsync(ref, vx, fbytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return fail_dev();
  best = 1e30f;
  SlabPlan bi = plan.inv;
  for (const SlabPlan& c : ci) {
    float ms = 0;
    if (timeit([&] { return inv(c); }, clear_vx, ms) != hipSuccess) return fail_dev();
    if (verify) {
      bool same = false;
      if (clear_vx() != hipSuccess || inv(c) != hipSuccess ||
          same_as_ref(vx, fbytes, same) != hipSuccess)
        return fail_dev();
      all_same = all_same && same;
    }
    if (ms < best) {
      best = ms;
      bi = c;
    }
  }
  release();
  if (!all_same) return KX_ERR_NUMERIC;
  plan.fwd = bf;
  plan.pen = bp;
  plan.inv = bi;
  ++g->gen;  // recorded graphs carry the old launch shapes
  kx_logf("autotune %s: fwd(qsplit %d, slabs %d, waves %d, kc %d, vlds %d) pen(waves %d, lds %zu, "
          "per %d) inv(slabs %d, waves %d, kc %d, vlds %d)",
          prec_name(prec), bf.qsplit, bf.slabs, bf.waves, bf.kc, bf.vlds ? 1 : 0, bp.waves,
          bp.lds_bytes, bp.per, bi.slabs, bi.waves, bi.kc, bi.vlds ? 1 : 0);
  if (cache_path && !verify) {
    if (FILE* f = std::fopen(cache_path, "a")) {
      std::fprintf(f, "%s | fwd %d %d %d %d %d %llu | pen %d %llu %d | inv %d %d %d %d %llu\n", key,
                   bf.qsplit, bf.slabs, bf.waves, bf.kc, bf.vlds ? 1 : 0,
                   (unsigned long long)bf.lds_bytes, bp.waves, (unsigned long long)bp.lds_bytes,
                   bp.per, bi.slabs, bi.waves, bi.kc, bi.vlds ? 1 : 0,
                   (unsigned long long)bi.lds_bytes);
      std::fclose(f);
    }
  }
  return KX_OK;
}

kx_status kx_get_plan(kx_grid* g, int prec, int* fwd_out, int* pen_out, int* inv_out) {
  if (!g || !fwd_out || !pen_out || !inv_out) return KX_ERR_INVALID_ARG;
  if (prec < KX_PREC_FP64 || prec > KX_PREC_MIXED) return KX_ERR_INVALID_ARG;
  Plan p = prec == KX_PREC_FP32
               ? g->plan_f
               : ((prec == KX_PREC_BF16X3 || prec == KX_PREC_FP16X3) ? g->plan_s : g->plan_d);
  if (prec == KX_PREC_MIXED) p.inv = g->plan_s.inv;
  const int f[6] = {p.fwd.qsplit, p.fwd.slabs, p.fwd.waves, p.fwd.kc, p.fwd.vlds ? 1 : 0,
                    (int)p.fwd.lds_bytes};
  const int q[3] = {p.pen.waves, (int)p.pen.lds_bytes, p.pen.per};
  const int v[6] = {1, p.inv.slabs, p.inv.waves, p.inv.kc, p.inv.vlds ? 1 : 0,
                    (int)p.inv.lds_bytes};
  std::copy(f, f + 6, fwd_out);
  std::copy(q, q + 3, pen_out);
  std::copy(v, v + 6, inv_out);
  return KX_OK;
}

kx_status kx_exchange_energy(kx_grid* g, double* ex_out) {
  if (!g || !ex_out) return KX_ERR_INVALID_ARG;
  if (g->last_norb < 0) return KX_ERR_STATE;
  double v = 0.0;
  if (hipMemcpyAsync(&v, g->dEx, sizeof(double), hipMemcpyDeviceToHost, g->stream) != hipSuccess ||
      hipStreamSynchronize(g->stream) != hipSuccess) {
    (void)hipGetLastError();
    return KX_ERR_DEVICE;
  }
  *ex_out = v;
  return KX_OK;
}

}  // extern "C"

namespace {

constexpr int kAceMaxOrb = 1024;   // one-workgroup Cholesky
constexpr int kAceMaxVec = 4096;

// grow a device buffer of doubles to at least n elements
kx_status ensure_doubles(kx_grid* g, double** p, long long* cap, long long n) {
  if (n <= *cap) return KX_OK;
  KX_HIP(hipStreamSynchronize(g->stream));
  dev_free(*p);
  *p = nullptr;
  *cap = 0;
  kx_status st = dev_alloc((void**)p, sizeof(double) * (size_t)n);
  if (st != KX_OK) return st;
  *cap = n;
  return KX_OK;
}

kx_status check_ace_fields(const kx_grid* g, int norb, int dtype, const void* a, const void* b,
                           const void* out) {
  if (!g || norb < 1 || norb > kAceMaxOrb || (long long)norb > g->geom.N) return KX_ERR_INVALID_ARG;
  if (dtype != KX_F64 && dtype != KX_F32) return KX_ERR_INVALID_ARG;
  if (!a || !b || !out || out == a || out == b) return KX_ERR_INVALID_ARG;
  return KX_OK;
}

// the compressed exchange's algebra on norb fields of N values of storage
// dtype (the real fields of a grid, or the real forms of complex fields)
kx_status ace_build_core(kx_grid* g, int norb, int dtype, long long N, const void* psi_dev,
                         const void* w_dev, void* xi_dev);
kx_status ace_apply_core(kx_grid* g, int norb, int dtype, long long N, const void* xi_dev, int nvec,
                         const void* phi_dev, void* out_dev);

}  // namespace

extern "C" {

kx_status kx_ace_build(kx_grid* g, int norb, int dtype, const void* psi_dev, const void* w_dev,
                       void* xi_dev) {
  const Range range("kx_ace_build");
  kx_status st = check_ace_fields(g, norb, dtype, psi_dev, w_dev, xi_dev);
  if (st != KX_OK) return st;
  return ace_build_core(g, norb, dtype, g->geom.N, psi_dev, w_dev, xi_dev);
}

kx_status kx_ace_build_complex(kx_grid* g, int norb, const void* psi_dev, const void* w_dev,
                               void* xi_dev) {
  const Range range("kx_ace_build_complex");
  if (!g || norb < 1 || 2 * norb > kAceMaxOrb || 2LL * norb > 2 * g->geom.N)
    return KX_ERR_INVALID_ARG;
  if (!psi_dev || !w_dev || !xi_dev || xi_dev == psi_dev || xi_dev == w_dev)
    return KX_ERR_INVALID_ARG;
  // the real forms [psi, i psi] and [W, i W]: 2 norb vectors of 2 N doubles each
  const long long N2 = 2 * g->geom.N, len = 2LL * norb * N2;
  kx_status st = ensure_doubles(g, &g->dAceU, &g->ace_u_cap, len);
  if (st == KX_OK) st = ensure_doubles(g, &g->dAceW, &g->ace_w_cap, len);
  if (st != KX_OK) return st;
  KX_HIP(launch_realify((const double*)psi_dev, norb, g->geom.N, g->dAceU, g->stream));
  KX_HIP(launch_realify((const double*)w_dev, norb, g->geom.N, g->dAceW, g->stream));
  return ace_build_core(g, 2 * norb, KX_F64, N2, g->dAceU, g->dAceW, xi_dev);
}

kx_status kx_ace_apply_complex(kx_grid* g, int norb, const void* xi_dev, int nvec,
                               const void* phi_dev, void* out_dev) {
  const Range range("kx_ace_apply_complex");
  if (!g || norb < 1 || 2 * norb > kAceMaxOrb) return KX_ERR_INVALID_ARG;
  if (!xi_dev || !phi_dev || !out_dev || out_dev == xi_dev || out_dev == phi_dev)
    return KX_ERR_INVALID_ARG;
  if (nvec < 1 || nvec > kAceMaxVec) return KX_ERR_INVALID_ARG;
  return ace_apply_core(g, 2 * norb, KX_F64, 2 * g->geom.N, xi_dev, nvec, phi_dev, out_dev);
}

}  // extern "C"

namespace {

kx_status ace_build_core(kx_grid* g, int norb, int dtype, long long N, const void* psi_dev,
                         const void* w_dev, void* xi_dev) {
  const long long nn = (long long)norb * norb;
  kx_status st;
  const long long grp = ace_groups(N, norb, norb);
  // partial sums for this build and for every later kx_ace_apply on up to
  // kAceMaxVec fields, and the apply's coefficients: kx_ace_apply allocates
  // nothing
  long long part = grp * nn;
  for (int nv = 1; nv <= kAceMaxVec; ++nv)
    part = std::max(part, ace_groups(N, norb, nv) * norb * (long long)nv);
  st = ensure_doubles(g, &g->dAcePart, &g->ace_part_cap, part);
  if (st != KX_OK) return st;
  st = ensure_doubles(g, &g->dAceG, &g->ace_g_cap, (long long)norb * kAceMaxVec);
  if (st != KX_OK) return st;
  if (nn > g->ace_mat_cap) {
    long long cap = g->ace_mat_cap;
    st = ensure_doubles(g, &g->dAceA, &cap, nn);
    if (st != KX_OK) return st;
    cap = g->ace_mat_cap;
    st = ensure_doubles(g, &g->dAceLinv, &cap, nn);
    if (st != KX_OK) return st;
    g->ace_mat_cap = nn;
  }
  if (!g->dAceStatus) {
    st = dev_alloc((void**)&g->dAceStatus, sizeof(int));
    if (st != KX_OK) return st;
  }
  const double dV = cell_dV(g);
  // -M = -(psi, W)_h, then its Cholesky factor and the factor's inverse
  KX_HIP(launch_gram(dtype, psi_dev, norb, w_dev, norb, N, grp, g->dAcePart, -dV, g->dAceA,
                     g->stream));
  KX_HIP(launch_chol_inv(g->dAceA, norb, g->dAceLinv, g->dAceStatus, g->stream));
  int fail = 0;
  KX_HIP(hipMemcpyAsync(&fail, g->dAceStatus, sizeof(int), hipMemcpyDeviceToHost, g->stream));
  KX_HIP(hipStreamSynchronize(g->stream));
  if (fail != 0) return KX_ERR_NUMERIC;
  g->ace_norb = std::max(g->ace_norb, norb);
  // xi = L^{-1} W
  KX_HIP(launch_combine(dtype, g->dAceLinv, norb, 1, norb, norb, w_dev, N, 1.0, xi_dev,
                        g->stream));
  return KX_OK;
}

kx_status ace_apply_core(kx_grid* g, int norb, int dtype, long long N, const void* xi_dev, int nvec,
                         const void* phi_dev, void* out_dev) {
  const long long nk = (long long)norb * nvec;
  const long long grp = ace_groups(N, norb, nvec);
  // buffers reserved by kx_ace_build
  if (norb > g->ace_norb || grp * nk > g->ace_part_cap || nk > g->ace_g_cap) return KX_ERR_STATE;
  const double dV = cell_dV(g);
  // G[k][v] = (xi_k, phi_v)_h, then out_v = -sum_k G[k][v] xi_k
  KX_HIP(launch_gram(dtype, xi_dev, norb, phi_dev, nvec, N, grp, g->dAcePart, dV, g->dAceG,
                     g->stream));
  KX_HIP(launch_combine(dtype, g->dAceG, 1, nvec, nvec, norb, xi_dev, N, -1.0, out_dev,
                        g->stream));
  return KX_OK;
}

}  // namespace

extern "C" {

kx_status kx_ace_apply(kx_grid* g, int norb, int dtype, const void* xi_dev, int nvec,
                       const void* phi_dev, void* out_dev) {
  const Range range("kx_ace_apply");
  kx_status st = check_ace_fields(g, norb, dtype, xi_dev, phi_dev, out_dev);
  if (st != KX_OK) return st;
  if (nvec < 1 || nvec > kAceMaxVec) return KX_ERR_INVALID_ARG;
  return ace_apply_core(g, norb, dtype, g->geom.N, xi_dev, nvec, phi_dev, out_dev);
}

kx_status kx_pair_energies(kx_grid* g, int npairs, const int* pairs_host, double* e_out_host) {
  if (!g || npairs < 0) return KX_ERR_INVALID_ARG;
  if (npairs > 0 && (!pairs_host || !e_out_host)) return KX_ERR_INVALID_ARG;
  if (g->last_norb < 0) return KX_ERR_STATE;
  const int norb = g->last_norb;
  for (int k = 0; k < npairs; ++k) {
    const int i = pairs_host[2 * k], j = pairs_host[2 * k + 1];
    if (i < 0 || j < 0 || i >= norb || j >= norb) return KX_ERR_INVALID_ARG;
  }
  if (npairs == 0) return KX_OK;
  const long long total = (long long)norb * (norb + 1) / 2;
  std::vector<double> all(total);
  if (hipStreamSynchronize(g->stream) != hipSuccess ||
      hipMemcpy(all.data(), g->last_pairE, sizeof(double) * total, hipMemcpyDeviceToHost) !=
          hipSuccess) {
    (void)hipGetLastError();
    return KX_ERR_DEVICE;
  }
  for (int k = 0; k < npairs; ++k) {
    const int i = std::min(pairs_host[2 * k], pairs_host[2 * k + 1]);
    const int j = std::max(pairs_host[2 * k], pairs_host[2 * k + 1]);
    e_out_host[k] = all[pair_index(i, j, norb)];
  }
  return KX_OK;
}

kx_status kx_get_eigensystem(kx_grid* g, int axis, double* lam_host, double* V_host) {
  if (!g || axis < 0 || axis > 2) return KX_ERR_INVALID_ARG;
  const int nk = g->n[axis];
  if (lam_host)
    for (int a = 0; a < nk; ++a) lam_host[a] = g->lam_host[axis][a];
  if (V_host)
    for (size_t idx = 0; idx < (size_t)nk * nk; ++idx) V_host[idx] = g->V_host[axis][idx];
  return KX_OK;
}

kx_status kx_profile(kx_grid* g, int enable) {
  if (!g || (enable != 0 && enable != 1)) return KX_ERR_INVALID_ARG;
  if (hipStreamSynchronize(g->stream) != hipSuccess) {
    (void)hipGetLastError();
    return KX_ERR_DEVICE;
  }
  g->prof_on = enable == 1;
  g->prof_mask = 0x1F;
  g->prof_kind.clear();
  return KX_OK;
}

kx_status kx_profile_phases(kx_grid* g, int mask) {
  if (!g || mask < 1 || mask > 0x1F) return KX_ERR_INVALID_ARG;
  if (hipStreamSynchronize(g->stream) != hipSuccess) {
    (void)hipGetLastError();
    return KX_ERR_DEVICE;
  }
  g->prof_on = true;
  g->prof_mask = mask;
  g->prof_kind.clear();
  return KX_OK;
}

kx_status kx_profile_read(kx_grid* g, int phase, double* total_ms, long long* launches) {
  if (!g || !total_ms || !launches || phase < 0 || phase > KX_PHASE_ACCUM) return KX_ERR_INVALID_ARG;
  if (hipStreamSynchronize(g->stream) != hipSuccess) {
    (void)hipGetLastError();
    return KX_ERR_DEVICE;
  }
  double tot = 0.0;
  long long cnt = 0;
  for (size_t k = 0; k < g->prof_kind.size(); ++k) {
    if (g->prof_kind[k] != phase) continue;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, g->prof_ev[2 * k], g->prof_ev[2 * k + 1]) != hipSuccess) {
      (void)hipGetLastError();
      return KX_ERR_DEVICE;
    }
    tot += ms;
    ++cnt;
  }
  *total_ms = tot;
  *launches = cnt;
  return KX_OK;
}

}  // extern "C"
