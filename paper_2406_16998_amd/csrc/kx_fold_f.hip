// Transform kernels instantiated for float MFMA operands (FP32 arithmetic), for
// double and float orbital storage.
#include "kx_fold.inc"

namespace kx {

hipError_t launch_forward_f(int storage, int mode, const Geom& g, const SlabPlan& p,
                               const EigR<float>& e, const void* src, const Item* items, int nitems,
                               float* T, hipStream_t s) {
  return storage == KX_F64
             ? fwd_launch<float, double>(mode, g, p, e, (const double*)src, items, nitems, T, s)
             : fwd_launch<float, float>(mode, g, p, e, (const float*)src, items, nitems, T, s);
}

hipError_t launch_pencil_f(const Geom& g, const PencilPlan& p, const EigR<float>& e,
                              const double* F, int nitems, float* T, double* epart, hipStream_t s) {
  return pen_launch<float, float>(g, p, e, F, nitems, T, T, epart, s);
}

hipError_t launch_inverse_f(int storage, int mode, const Geom& g, const SlabPlan& p,
                               const EigR<float>& e, const float* T, const Item* items, int nitems,
                               const void* psi, const double* occ, void* dst, hipStream_t s) {
  return storage == KX_F64
             ? inv_launch<float, double>(mode, g, p, e, T, items, nitems, (const double*)psi, occ,
                                      (double*)dst, s)
             : inv_launch<float, float>(mode, g, p, e, T, items, nitems, (const float*)psi, occ,
                                     (float*)dst, s);
}

}  // namespace kx
