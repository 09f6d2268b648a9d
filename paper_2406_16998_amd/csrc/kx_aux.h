// Internal declarations of auxiliary kernels outside the transform passes
// (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

namespace kx {

// The compressed exchange of complex fields runs the real algebra on their
// real form: a complex field of N values, interleaved (re, im), is a real
// vector of 2 N values, and the real form of the span of n complex fields is
// spanned by the 2 n real vectors {z_j, i z_j}.  dst (2 n vectors of 2 N
// doubles) = [src_0 .. src_{n-1}, i src_0 .. i src_{n-1}].
hipError_t launch_realify(const double* src, int n, long long N, double* dst, hipStream_t s);

}  // namespace kx
