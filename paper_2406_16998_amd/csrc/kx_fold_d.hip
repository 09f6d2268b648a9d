// Transform kernels instantiated for double MFMA operands (FP64 arithmetic), for
// double and float orbital storage.
#include "kx_fold.inc"

namespace kx {

hipError_t launch_forward_d(int storage, int mode, const Geom& g, const SlabPlan& p,
                               const EigR<double>& e, const void* src, const Item* items, int nitems,
                               double* T, hipStream_t s) {
  return storage == KX_F64
             ? fwd_launch<double, double>(mode, g, p, e, (const double*)src, items, nitems, T, s)
             : fwd_launch<double, float>(mode, g, p, e, (const float*)src, items, nitems, T, s);
}

hipError_t launch_pencil_d(const Geom& g, const PencilPlan& p, const EigR<double>& e,
                              const double* F, int nitems, double* T, double* epart, hipStream_t s,
                              float* out_f) {
  return out_f ? pen_launch<double, float>(g, p, e, F, nitems, T, out_f, epart, s)
               : pen_launch<double, double>(g, p, e, F, nitems, T, T, epart, s);
}

hipError_t launch_pencil_half(int dir, const Geom& g, const EigR<double>& e, int nitems, double* T,
                              double* S, hipStream_t s) {
  return half_launch(dir, g, e, nitems, T, S, s);
}

hipError_t launch_inverse_d(int storage, int mode, const Geom& g, const SlabPlan& p,
                               const EigR<double>& e, const double* T, const Item* items, int nitems,
                               const void* psi, const double* occ, void* dst, hipStream_t s) {
  return storage == KX_F64
             ? inv_launch<double, double>(mode, g, p, e, T, items, nitems, (const double*)psi, occ,
                                      (double*)dst, s)
             : inv_launch<double, float>(mode, g, p, e, T, items, nitems, (const float*)psi, occ,
                                     (float*)dst, s);
}

}  // namespace kx
