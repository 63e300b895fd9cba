// k_lorenzo.hip -- first-order Lorenzo alternative (Sec. 6.5), gfx950.
//
// Dual quantization: every value is first rounded to the nearest multiple of
// 2e (the integer v = round(x / 2e), half away from zero, in double); the code
// is the integer residual delta = v - L(v) of the first-order Lorenzo
// predictor over the dimensions of size > 1 (outside the grid counts as 0),
// i.e. the mixed first difference of v.  Each thread computes its residual
// directly by inclusion-exclusion over its 2^D lower neighbours, so compression
// has no sequential dependency.  Decompression rebuilds v by running sums
// along every dimension and outputs (T)(v * 2e); the rare points where that
// misses the bound are patched verbatim.

#include "interp_dev.h"
#include "lorenzo_dev.h"

namespace hpez {

constexpr double kPreqLimit = 4503599627370496.0;  // 2^52

template <typename T>
__device__ __forceinline__ long long preq(T x, double inv2e, bool& bad)
{
  const double t = (double)x * inv2e;
  const double qf = floor(fabs(t) + 0.5);
  if (!(qf < kPreqLimit)) {
    bad = true;
    return 0;
  }
  return (long long)(t < 0 ? -qf : qf);
}

template <typename T>
__device__ __forceinline__ long long residual(const T* __restrict__ X, const Geom& g, int64_t i,
                                              const int64_t* x, double inv2e, bool& bad)
{
  long long delta = 0;
  for (unsigned S = 0; S < 16; S++) {
    int64_t j = i;
    bool in = true;
    for (int d = 0; d < 4; d++)
      if (S >> d & 1u) {
        if (x[d] == 0) in = false;
        j -= g.st[d];
      }
    if (!in) continue;
    const long long v = preq<T>(X[j], inv2e, bad);
    delta += (__popc(S) & 1) ? -v : v;
  }
  return delta;
}

__device__ __forceinline__ void coords(const Geom& g, int64_t i, int64_t* x)
{
  int64_t r = i;
  for (int d = 3; d >= 0; d--) {
    x[d] = r % g.n[d];
    r /= g.n[d];
  }
}

template <typename T>
__device__ __forceinline__ bool misses(T xv, long long v, double twoe, double e)
{
  const T xr = (T)((double)v * twoe);
  return !(fabs((double)xr - (double)xv) <= e);
}

template <typename T>
__global__ void __launch_bounds__(256) lorenzo_code_kernel(const T* __restrict__ X, Geom g, uint64_t n,
                                                           LorenzoArgs a, uint16_t* __restrict__ code,
                                                           uint32_t* __restrict__ pcount,
                                                           int* __restrict__ bad_flag)
{
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    int64_t x[4];
    coords(g, (int64_t)i, x);
    bool bad = false;
    const long long delta = residual<T>(X, g, (int64_t)i, x, a.inv2e, bad);
    const long long v = preq<T>(X[i], a.inv2e, bad);
    if (bad) atomicOr(bad_flag, 1);
    const long long R = a.R;
    code[brick_pos(g.n, x)] = (delta > -R && delta < R) ? (uint16_t)(delta + R) : (uint16_t)0;
    if (!bad && misses<T>(X[i], v, a.twoe, a.e)) atomicAdd(&pcount[i / a.chunk], 1u);
  }
}

// outlier residuals (code 0) and patches, in row-major order, chunk by chunk
template <typename T>
__global__ void __launch_bounds__(256) lorenzo_gather_kernel(
    const T* __restrict__ X, Geom g, uint64_t n, LorenzoArgs a, const uint16_t* __restrict__ code,
    const uint32_t* __restrict__ czero, const uint64_t* __restrict__ zoff,
    const uint32_t* __restrict__ pcount, const uint64_t* __restrict__ poff,
    long long* __restrict__ outl, uint64_t* __restrict__ pidx, T* __restrict__ pval, uint64_t nch)
{
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nch || (czero[k] == 0 && pcount[k] == 0)) return;
  const uint64_t beg = k * a.chunk;
  const uint64_t end = beg + a.chunk < n ? beg + a.chunk : n;
  // outliers: chunk k of the stream order
  if (czero[k]) {
    uint64_t z = zoff[k];
    for (uint64_t i = beg; i < end; i++) {
      if (code[i] != 0) continue;
      int64_t x[4];
      bool bad = false;
      brick_coords(g.n, (int64_t)i, x);
      const int64_t r = x[0] * g.st[0] + x[1] * g.st[1] + x[2] * g.st[2] + x[3];
      outl[z++] = residual<T>(X, g, r, x, a.inv2e, bad);
    }
  }
  // patches: chunk k of the row-major order
  if (pcount[k]) {
    uint64_t p = poff[k];
    for (uint64_t i = beg; i < end; i++) {
      bool bad = false;
      const long long v = preq<T>(X[i], a.inv2e, bad);
      if (misses<T>(X[i], v, a.twoe, a.e)) {
        pidx[p] = i;
        pval[p] = X[i];
        p++;
      }
    }
  }
}

// decompression: residuals from codes and outliers
__global__ void __launch_bounds__(256) lorenzo_delta_kernel(const uint16_t* __restrict__ code, uint64_t n,
                                                            uint32_t R, long long* __restrict__ v,
                                                            Geom g)
{
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    int64_t x[4];
    coords(g, (int64_t)i, x);
    const uint32_t c = code[brick_pos(g.n, x)];
    v[i] = c ? (long long)c - (long long)R : 0;
  }
}

__global__ void __launch_bounds__(256) lorenzo_outlier_kernel(
    const uint16_t* __restrict__ code, uint64_t n, uint32_t chunk, const uint32_t* __restrict__ czero,
    const uint64_t* __restrict__ zoff, const long long* __restrict__ outl, uint64_t n_outl,
    long long* __restrict__ v, int* __restrict__ status, uint64_t nch, Geom g)
{
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nch || czero[k] == 0) return;
  const uint64_t beg = k * chunk;
  const uint64_t end = beg + chunk < n ? beg + chunk : n;
  uint64_t z = zoff[k];
  for (uint64_t i = beg; i < end; i++) {
    if (code[i] != 0) continue;
    if (z >= n_outl) {
      atomicOr(status, 1);
      return;
    }
    int64_t x[4];
    brick_coords(g.n, (int64_t)i, x);
    v[x[0] * g.st[0] + x[1] * g.st[1] + x[2] * g.st[2] + x[3]] = outl[z++];
  }
}

// running sums along a non-fastest dimension: one thread per line, lines of
// consecutive threads are adjacent in memory
__global__ void __launch_bounds__(256) integrate_kernel(long long* __restrict__ v, int64_t len,
                                                        int64_t st, uint64_t lines)
{
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t L = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; L < lines; L += stride) {
    const uint64_t outer = L / (uint64_t)st, inner = L % (uint64_t)st;
    long long* p = v + outer * (uint64_t)len * (uint64_t)st + inner;
    long long acc = p[0];
    for (int64_t x = 1; x < len; x++) {
      acc += p[x * st];
      p[x * st] = acc;
    }
  }
}

// running sums along the fastest dimension: one wavefront per row
__global__ void __launch_bounds__(256) integrate_rows_kernel(long long* __restrict__ v, int64_t len,
                                                             uint64_t rows)
{
  const uint64_t wid = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (wid >= rows) return;
  long long* p = v + wid * (uint64_t)len;
  long long carry = 0;
  for (int64_t base = 0; base < len; base += 64) {
    const int64_t i = base + lane;
    long long x = i < len ? p[i] : 0;
    for (int o = 1; o < 64; o <<= 1) {
      const long long y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    x += carry;
    if (i < len) p[i] = x;
    carry = __shfl(x, 63, 64);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) lorenzo_output_kernel(const long long* __restrict__ v, uint64_t n,
                                                             double twoe, T* __restrict__ out)
{
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = (T)((double)v[i] * twoe);
}

template <typename T>
__global__ void __launch_bounds__(256) patch_kernel(const uint64_t* __restrict__ pidx,
                                                    const T* __restrict__ pval, uint64_t np,
                                                    uint64_t n, T* __restrict__ out,
                                                    int* __restrict__ status)
{
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= np) return;
  const uint64_t i = pidx[k];
  if (i >= n) {
    atomicOr(status, 1);
    return;
  }
  out[i] = pval[k];
}

static unsigned gridn(uint64_t n)
{
  uint64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  return (unsigned)(b ? b : 1);
}

template <typename T>
hipError_t launch_lorenzo_codes(const T* X, const Geom& g, uint64_t n, const LorenzoArgs& a,
                                uint16_t* code, uint32_t* pcount, int* bad, hipStream_t st)
{
  if (!n) return hipSuccess;
  hipLaunchKernelGGL((lorenzo_code_kernel<T>), dim3(gridn(n)), dim3(256), 0, st, X, g, n, a, code,
                     pcount, bad);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_lorenzo_gather(const T* X, const Geom& g, uint64_t n, const LorenzoArgs& a,
                                 const uint16_t* code, const uint32_t* czero, const uint64_t* zoff,
                                 const uint32_t* pcount, const uint64_t* poff, long long* outl,
                                 uint64_t* pidx, T* pval, hipStream_t st)
{
  const uint64_t nch = (n + a.chunk - 1) / a.chunk;
  if (!nch) return hipSuccess;
  hipLaunchKernelGGL((lorenzo_gather_kernel<T>), dim3((unsigned)((nch + 255) / 256)), dim3(256), 0,
                     st, X, g, n, a, code, czero, zoff, pcount, poff, outl, pidx, pval, nch);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_lorenzo_rebuild(const uint16_t* code, const Geom& g, uint64_t n, uint32_t R,
                                  uint32_t chunk, const uint32_t* czero, const uint64_t* zoff,
                                  const long long* outl, uint64_t n_outl, const uint64_t* pidx,
                                  const T* pval, uint64_t n_patch, double twoe, long long* v,
                                  T* out, int* status, hipStream_t st)
{
  if (!n) return hipSuccess;
  const uint64_t nch = (n + chunk - 1) / chunk;
  hipLaunchKernelGGL(lorenzo_delta_kernel, dim3(gridn(n)), dim3(256), 0, st, code, n, R, v, g);
  hipLaunchKernelGGL(lorenzo_outlier_kernel, dim3((unsigned)((nch + 255) / 256)), dim3(256), 0, st,
                     code, n, chunk, czero, zoff, outl, n_outl, v, status, nch, g);
  for (int d = 0; d < 4; d++) {
    if (g.n[d] <= 1) continue;
    if (g.st[d] == 1) {
      const uint64_t rows = n / (uint64_t)g.n[d];
      hipLaunchKernelGGL(integrate_rows_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, v,
                         g.n[d], rows);
    } else {
      const uint64_t lines = n / (uint64_t)g.n[d];
      hipLaunchKernelGGL(integrate_kernel, dim3(gridn(lines)), dim3(256), 0, st, v, g.n[d], g.st[d],
                         lines);
    }
  }
  hipLaunchKernelGGL((lorenzo_output_kernel<T>), dim3(gridn(n)), dim3(256), 0, st, v, n, twoe, out);
  if (n_patch)
    hipLaunchKernelGGL((patch_kernel<T>), dim3((unsigned)((n_patch + 255) / 256)), dim3(256), 0, st,
                       pidx, pval, n_patch, n, out, status);
  return hipGetLastError();
}

#define INST(T)                                                                                  \
  template hipError_t launch_lorenzo_codes<T>(const T*, const Geom&, uint64_t, const LorenzoArgs&, \
                                              uint16_t*, uint32_t*, int*, hipStream_t);          \
  template hipError_t launch_lorenzo_gather<T>(const T*, const Geom&, uint64_t,                  \
                                               const LorenzoArgs&, const uint16_t*,              \
                                               const uint32_t*, const uint64_t*, const uint32_t*, \
                                               const uint64_t*, long long*, uint64_t*, T*,       \
                                               hipStream_t);                                     \
  template hipError_t launch_lorenzo_rebuild<T>(const uint16_t*, const Geom&, uint64_t, uint32_t, \
                                                uint32_t, const uint32_t*, const uint64_t*,      \
                                                const long long*, uint64_t, const uint64_t*,     \
                                                const T*, uint64_t, double, long long*, T*, int*, \
                                                hipStream_t);
INST(float)
INST(double)

}  // namespace hpez
