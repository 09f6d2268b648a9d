// Deterministic energy reductions and the launch-shape planner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "kx_internal.h"

namespace kx {
namespace {
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

// elementwise precision conversion, 4 elements a thread per step
__global__ void __launch_bounds__(256) narrow_kernel(const double* __restrict__ a, float* __restrict__ b,
                                                     long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x * 4;
  for (long long k = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * 4; k < n; k += stride) {
    if (k + 3 < n) {
      const double2 u = *reinterpret_cast<const double2*>(a + k);
      const double2 v = *reinterpret_cast<const double2*>(a + k + 2);
      *reinterpret_cast<float4*>(b + k) = make_float4((float)u.x, (float)u.y, (float)v.x, (float)v.y);
    } else {
      for (long long m = k; m < n; ++m) b[m] = (float)a[m];
    }
  }
}

__global__ void __launch_bounds__(256) widen_kernel(const float* __restrict__ a, double* __restrict__ b,
                                                    long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x * 4;
  for (long long k = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * 4; k < n; k += stride) {
    if (k + 3 < n) {
      const float4 u = *reinterpret_cast<const float4*>(a + k);
      *reinterpret_cast<double2*>(b + k) = make_double2(u.x, u.y);
      *reinterpret_cast<double2*>(b + k + 2) = make_double2(u.z, u.w);
    } else {
      for (long long m = k; m < n; ++m) b[m] = a[m];
    }
  }
}

__global__ void __launch_bounds__(256) zero_kernel(unsigned* __restrict__ p, long long words,
                                                   int vec) {
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nthr = (long long)gridDim.x * blockDim.x;
  long long done = 0;
  if (vec) {
    const long long quads = words / 4;
    uint4* q = reinterpret_cast<uint4*>(p);
    for (long long k = tid; k < quads; k += nthr) q[k] = make_uint4(0u, 0u, 0u, 0u);
    done = quads * 4;
  }
  for (long long k = done + tid; k < words; k += nthr) p[k] = 0u;
}

// deterministic values in [-1, 1) from the element index (tuning inputs)
__global__ void __launch_bounds__(256) pattern_kernel(void* __restrict__ p, long long n, int dbl) {
  const long long nthr = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += nthr) {
    unsigned long long x = (unsigned long long)k * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    x ^= x >> 29;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 32;
    const double v = (double)(x >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    if (dbl)
      static_cast<double*>(p)[k] = v;
    else
      static_cast<float*>(p)[k] = (float)v;
  }
}

// number of 32-bit words that differ between a and b
__global__ void __launch_bounds__(256) diff_kernel(const unsigned* __restrict__ a,
                                                   const unsigned* __restrict__ b, long long words,
                                                   unsigned long long* __restrict__ count) {
  const long long nthr = (long long)gridDim.x * blockDim.x;
  unsigned long long c = 0;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < words; k += nthr)
    c += a[k] != b[k];
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

// diagonal pairs at [0, norb); round r of the tournament at norb + r c,
// c = floor(norb / 2) real pairs per round (the dummy's pair is skipped)
__global__ void __launch_bounds__(256) schedule_kernel(int norb, Item* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = (norb + 1) & ~1;
  const int c = norb / 2;
  if (t < norb) out[t] = Item{t, t};
  if (t < m - 1) {
    Item* __restrict__ o = out + norb + (long long)t * c;
    int n = 0;
    for (int k = 0; k < m / 2; ++k) {
      const Item p = rr_pair(m, t, k);
      if (p.j < norb) o[n++] = p;
    }
  }
}

__global__ void __launch_bounds__(256) field_items_kernel(int n, Item* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n) out[b] = Item{b, -1};
}

constexpr int kPutVals = 64;  // doubles per launch: 512 bytes of kernel arguments
struct PutVals {
  double v[kPutVals];
};
__global__ void __launch_bounds__(64) put_doubles_kernel(PutVals vals, int n,
                                                        double* __restrict__ dst) {
  const int k = threadIdx.x;
  if (k < n) dst[k] = vals.v[k];
}

}  // namespace

hipError_t launch_schedule(int norb, Item* out, hipStream_t s) {
  if (norb <= 0) return hipSuccess;
  const int m = (norb + 1) & ~1;
  const int t = norb > m - 1 ? norb : m - 1;
  hipLaunchKernelGGL(schedule_kernel, dim3((t + 255) / 256), dim3(256), 0, s, norb, out);
  return hipGetLastError();
}

hipError_t launch_field_items(int n, Item* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(field_items_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, out);
  return hipGetLastError();
}

hipError_t launch_put_doubles(const double* vals, int n, double* dst, hipStream_t s) {
  for (int k0 = 0; k0 < n; k0 += kPutVals) {
    PutVals pv;
    const int cnt = n - k0 < kPutVals ? n - k0 : kPutVals;
    for (int k = 0; k < kPutVals; ++k) pv.v[k] = k < cnt ? vals[k0 + k] : 0.0;
    hipLaunchKernelGGL(put_doubles_kernel, dim3(1), dim3(64), 0, s, pv, cnt, dst + k0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_pattern(void* p, long long n, bool dbl, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long blocks = std::max<long long>(1, std::min<long long>((n + 255) / 256, 8192));
  hipLaunchKernelGGL(pattern_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, dbl ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_diff(const void* a, const void* b, size_t bytes, unsigned long long* count,
                       hipStream_t s) {
  if (bytes % 4 != 0) return hipErrorInvalidValue;
  const long long words = (long long)(bytes / 4);
  if (words == 0) return hipSuccess;
  const long long blocks = std::max<long long>(1, std::min<long long>((words + 255) / 256, 8192));
  hipLaunchKernelGGL(diff_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (const unsigned*)a,
                     (const unsigned*)b, words, count);
  return hipGetLastError();
}

void allow_dynamic_lds(const void* fn, size_t lds) {
  if (lds <= 64 * 1024) return;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    dev = 0;
  }
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, size_t> done;
  std::lock_guard<std::mutex> lock(mu);
  size_t& set = done[{fn, dev}];
  if (set >= lds) return;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess)
    set = lds;
  else
    (void)hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if (bytes % 4 != 0 || (reinterpret_cast<uintptr_t>(p) % 4) != 0) return hipErrorInvalidValue;
  const long long words = (long long)(bytes / 4);
  const int vec = (reinterpret_cast<uintptr_t>(p) % 16) == 0;
  const long long blocks = std::max<long long>(1, std::min<long long>((words + 1023) / 1024, 8192));
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (unsigned*)p, words, vec);
  return hipGetLastError();
}

namespace {
// flag[0] = 1 if any of x[0 .. n) is NaN or infinite (every writer stores 1)
template <class S>
__global__ void __launch_bounds__(256) nonfinite_kernel(const S* __restrict__ x, long long n,
                                                       unsigned* __restrict__ flag) {
  bool bad = false;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x)
    bad = bad || !isfinite(x[k]);
  if (bad) flag[0] = 1u;
}
}  // namespace

hipError_t launch_nonfinite(const void* x, int storage, long long n, unsigned* flag, hipStream_t s) {
  hipError_t e = launch_zero(flag, sizeof(unsigned), s);
  if (e != hipSuccess || n <= 0) return e;
  const long long blocks = std::max<long long>(1, std::min<long long>((n + 255) / 256, 8192));
  if (storage == KX_F64)
    hipLaunchKernelGGL(nonfinite_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const double*)x, n, flag);
  else
    hipLaunchKernelGGL(nonfinite_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const float*)x, n, flag);
  return hipGetLastError();
}

hipError_t launch_narrow(const double* a, float* b, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long blocks = std::min<long long>((n + 1023) / 1024, 8192);
  hipLaunchKernelGGL(narrow_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}

hipError_t launch_widen(const float* a, double* b, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long blocks = std::min<long long>((n + 1023) / 1024, 8192);
  hipLaunchKernelGGL(widen_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}

// ================================================================ planning
Plan make_plan(const Geom& g, size_t max_lds, size_t esize) {
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
    const size_t vb = (size_t)(f.qsplit == 1 ? g.pe1 * g.pe1 + g.po1 * g.po1 : g.pe1 * g.pe1) * esize;
    // the largest chunk whose staging fits (V1 blocks in LDS if possible)
    f.kc = 0;
    for (size_t extra : {vb, (size_t)0}) {
      for (int c : {16, 8, 4}) {
        // register staging: every staged position of a chunk has a register slot
        if (c > fwd_max_kc(esize) || (esize != 8 && (size_t)c * g.pe1 > (size_t)kFwdPos * wps * 64))
          continue;
        if ((size_t)f.slabs * fwd_slab_bytes(g, c, wrow, esize) + extra <= max_lds) {
          f.kc = c;
          break;
        }
      }
      if (f.kc) break;
    }
    f.ok = f.kc != 0;
    if (!f.ok) f.kc = 4;
    const size_t chunk = (size_t)f.slabs * fwd_slab_bytes(g, f.kc, wrow, esize);
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
    const size_t vb = (size_t)(g.pe2 * g.pe2 + g.po2 * g.po2) * esize;
    v.kc = inv_kc(esize);
    auto chunks = [&](int sl) { return (size_t)sl * inv_slab_elems(g, v.kc, inv_band(esize)) * esize; };
    while (v.slabs > 1 && chunks(v.slabs) > max_lds) --v.slabs;
    v.waves = v.slabs * wps;
    v.ok = chunks(v.slabs) <= max_lds;
    v.vlds = chunks(v.slabs) + vb <= max_lds;
    v.lds_bytes = chunks(v.slabs) + (v.vlds ? vb : 0);
  }
  {
    PencilPlan& p = pl.pen;
    p.waves = 8;
    const size_t vb = (size_t)(g.pe3 * (g.pe3 + 1) + g.po3 * (g.po3 + 1)) * esize;
    p.lds_bytes = vb <= max_lds ? vb : 0;
  }
  return pl;
}

// ---------------------------------------------------------------- tuning
// Every launch shape the transform kernels accept for this grid (kind 0:
// double operands, 1: float operands, 2: split-BF16), each within the
// kernels' launch bounds, register staging budgets and the LDS size.
void plan_candidates(const Geom& g, size_t max_lds, int kind, std::vector<SlabPlan>& fwd,
                     std::vector<PencilPlan>& pen, std::vector<SlabPlan>& inv, size_t ssize) {
  fwd.clear();
  pen.clear();
  inv.clear();
  const size_t esize = kind == 0 ? sizeof(double) : sizeof(float);
  const bool split = kind == 2;
  const int ntx = g.pe1 / kTile, nty = g.pe2 / kTile, ntz = g.pe3 / kTile;
  {
    const int maxw = fwd_mt(ntx) / 64;
    for (int qsplit : {1, 2}) {
      const int wps = (qsplit == 1 ? 2 : 1) * (g.p2 / kTile);
      if (wps > maxw) continue;
      const int wrow = qsplit == 1 ? g.p1 : g.pe1;
      const size_t vb =
          (size_t)(qsplit == 1 ? g.pe1 * g.pe1 + g.po1 * g.po1 : g.pe1 * g.pe1) * esize;
      for (int slabs : {1, 2, 4, 8}) {
        if (slabs * wps > maxw) continue;
        for (int kc : {4, 8, 16}) {
          if (split ? kc != 16 : kc > fwd_max_kc(esize)) continue;
          if (!split && esize != 8 && (size_t)kc * g.pe1 > (size_t)kFwdPos * wps * 64) continue;
          for (int vl : {0, 1}) {
            if (split && vl) continue;
            const size_t lds8 = split ? (size_t)slabs * 2 * 2 * kc * wrow * esize
                                      : (size_t)slabs * fwd_slab_bytes(g, kc, wrow, esize) +
                                            (vl ? vb : 0);
            if (lds8 > max_lds) continue;  // launchable for 8-byte storage too
            const size_t lds = split ? lds8
                                     : (size_t)slabs * fwd_slab_bytes(g, kc, wrow, esize, ssize) +
                                           (vl ? vb : 0);
            SlabPlan p;
            p.qsplit = qsplit;
            p.slabs = slabs;
            p.waves = slabs * wps;
            p.kc = kc;
            p.vlds = vl != 0;
            p.lds_bytes = lds;
            fwd.push_back(p);
          }
        }
      }
    }
  }
  {
    const int maxw = pen_mt(ntz) / 64;
    const size_t vb = (size_t)(g.pe3 * (g.pe3 + 1) + g.po3 * (g.po3 + 1)) * esize;
    for (int w : {2, 4, 8, 16}) {
      if (w > maxw) continue;
      for (int vl : {0, 1}) {
        if ((split && vl) || (vl && vb > max_lds)) continue;
        PencilPlan p;
        p.waves = w;
        p.lds_bytes = vl ? vb : 0;
        pen.push_back(p);
      }
    }
    // split pencils: the pre-split V3 planes in LDS
    if (split && spen_vbytes(g) <= max_lds) {
      for (int w : {2, 4, 8, 16}) {
        if (w > maxw) continue;
        PencilPlan p;
        p.waves = w;
        p.lds_bytes = spen_vbytes(g);
        pen.push_back(p);
      }
    }
    // the pipelined pencil (V3 in LDS, two waves per SIMD, several items per wave)
    if (!split && ntz <= kPipeMaxNT && vb <= max_lds) {
      for (int w : {4, 8}) {
        for (int per : {2, 4, 8, 16}) {
          PencilPlan p;
          p.waves = w;
          p.lds_bytes = vb;
          p.per = per;
          pen.push_back(p);
        }
      }
    }
  }
  {
    const int maxw = inv_mt(nty) / 64;
    const int wps = g.pe1 / kTile;
    const size_t vb = (size_t)(g.pe2 * g.pe2 + g.po2 * g.po2) * esize;
    for (int slabs = 1; slabs * wps <= maxw; ++slabs) {
      for (int kc : {4, 8, 16}) {
        if (kc != inv_kc(esize)) continue;  // chunks are copied in 1 KB segments
        for (int vl : {0, 1}) {
          // split: the pre-split V2 blocks (three bf16 planes, padded rows)
          const size_t lds = split ? split_inv_lds(g, slabs, vl != 0)
                                   : (size_t)slabs * inv_slab_elems(g, kc, inv_band(esize)) * esize + (vl ? vb : 0);
          if (lds > max_lds) continue;
          SlabPlan p;
          p.slabs = slabs;
          p.waves = slabs * wps;
          p.kc = kc;
          p.vlds = vl != 0;
          p.lds_bytes = lds;
          inv.push_back(p);
        }
      }
    }
    // FP64 operands: the b parities on separate waves, twice the waves a slab
    if (kind == 0) {
      const int maxb = inv_bsplit_mt(nty) / 64;
      for (int slabs = 1; 2 * slabs * wps <= maxb; ++slabs) {
        for (int vl : {0, 1}) {
          const size_t lds =
              (size_t)slabs * inv_slab_elems(g, inv_kc(esize), true) * esize + (vl ? vb : 0);
          if (lds > max_lds) continue;
          SlabPlan p;
          p.slabs = slabs;
          p.waves = 2 * slabs * wps;
          p.kc = inv_kc(esize);
          p.vlds = vl != 0;
          p.lds_bytes = lds;
          inv.push_back(p);
        }
      }
    }
  }
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
