// k_convert.hip -- integer fields to float64 and back.  The method runs in
// double on an integer field's values (each rebuilt value rounded to an
// integer); the reconstruction returns to the field's type clamped to its
// range, which can only move a value toward the original (itself in range),
// so the point-wise bound still holds.
#include "hpez_host.h"
#include "hpez_internal.h"

namespace hpez {
namespace {

template <typename I>
__global__ void __launch_bounds__(256) to_f64_kernel(const I* __restrict__ in, double* __restrict__ out,
                                                     uint64_t n)
{
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = (double)in[i];
}

template <typename I>
__global__ void __launch_bounds__(256) from_f64_kernel(const double* __restrict__ in, I* __restrict__ out,
                                                       uint64_t n, double lo, double hi)
{
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double v = in[i];
    out[i] = (I)(v < lo ? lo : (v > hi ? hi : v));
  }
}

unsigned grid_of(uint64_t n)
{
  uint64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  return (unsigned)(b ? b : 1);
}

template <typename I>
hipError_t to_f64(const void* in, double* out, uint64_t n, hipStream_t st)
{
  hipLaunchKernelGGL(to_f64_kernel<I>, dim3(grid_of(n)), dim3(256), 0, st, (const I*)in, out, n);
  return hipGetLastError();
}

template <typename I>
hipError_t from_f64(const double* in, void* out, uint64_t n, double lo, double hi, hipStream_t st)
{
  hipLaunchKernelGGL(from_f64_kernel<I>, dim3(grid_of(n)), dim3(256), 0, st, in, (I*)out, n, lo, hi);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_int_to_f64(const void* in, int dt, double* out, uint64_t n, hipStream_t st)
{
  if (!n) return hipSuccess;
  switch (dt) {
    case HPEZ_U8: return to_f64<uint8_t>(in, out, n, st);
    case HPEZ_U16: return to_f64<uint16_t>(in, out, n, st);
    case HPEZ_I16: return to_f64<int16_t>(in, out, n, st);
    case HPEZ_I32: return to_f64<int32_t>(in, out, n, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_f64_to_int(const double* in, int dt, void* out, uint64_t n, hipStream_t st)
{
  if (!n) return hipSuccess;
  switch (dt) {
    case HPEZ_U8: return from_f64<uint8_t>(in, out, n, 0.0, 255.0, st);
    case HPEZ_U16: return from_f64<uint16_t>(in, out, n, 0.0, 65535.0, st);
    case HPEZ_I16: return from_f64<int16_t>(in, out, n, -32768.0, 32767.0, st);
    case HPEZ_I32: return from_f64<int32_t>(in, out, n, -2147483648.0, 2147483647.0, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hpez
