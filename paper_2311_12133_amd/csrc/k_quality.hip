// k_quality.hip -- reductions for the quality functions M of Sec. 3.1, Eq. (1):
// value range, maximum error, mean squared error (PSNR) and windowed SSIM of a
// reconstruction.  Every sum runs in a fixed order (per-thread strided
// partials, work-group trees, then one work-group over the partials in index
// order), so a result depends only on the inputs and the grid, which the host
// derives from the sizes alone.
#include "quality_dev.h"

namespace hpez {

namespace {

// fixed-order sum over the work-group (tree in LDS); thread 0 gets the total
template <int NT>
__device__ __forceinline__ double wg_sum(double v, double* red)
{
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double t = red[0];
  __syncthreads();
  return t;
}

template <int NT>
__device__ __forceinline__ double wg_max(double v, double* red)
{
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  const double t = red[0];
  __syncthreads();
  return t;
}

template <int NT>
__device__ __forceinline__ double wg_min(double v, double* red)
{
  return -wg_max<NT>(-v, red);
}

constexpr int kQT = 256;  // threads per work-group of the reductions

// Per work-group partials over points [g * per, (g + 1) * per): sum of
// squared errors, max |error|, min and max of x.
template <typename T>
__global__ void __launch_bounds__(kQT) qsum_kernel(const T* __restrict__ x, const T* __restrict__ xr,
                                                   uint64_t n, uint64_t per, double* __restrict__ part)
{
  __shared__ double red[kQT];
  const uint64_t b = (uint64_t)blockIdx.x * per;
  const uint64_t e = b + per < n ? b + per : n;
  double sse = 0.0, mx_err = 0.0, lo = INFINITY, hi = -INFINITY;
  for (uint64_t i = b + threadIdx.x; i < e; i += kQT) {
    const double a = (double)x[i], r = (double)xr[i];
    const double d = a - r;
    sse += d * d;
    mx_err = fmax(mx_err, fabs(d));
    lo = fmin(lo, a);
    hi = fmax(hi, a);
  }
  sse = wg_sum<kQT>(sse, red);
  mx_err = wg_max<kQT>(mx_err, red);
  lo = wg_min<kQT>(lo, red);
  hi = wg_max<kQT>(hi, red);
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x + 0] = sse;
    part[4 * blockIdx.x + 1] = mx_err;
    part[4 * blockIdx.x + 2] = lo;
    part[4 * blockIdx.x + 3] = hi;
  }
}

// one work-group: the partials of qsum_kernel in index order
__global__ void __launch_bounds__(kQT) qsum_final_kernel(const double* __restrict__ part, uint32_t np,
                                                         double* __restrict__ out)
{
  __shared__ double red[kQT];
  double sse = 0.0, mx_err = 0.0, lo = INFINITY, hi = -INFINITY;
  for (uint32_t i = threadIdx.x; i < np; i += kQT) {
    sse += part[4 * i + 0];
    mx_err = fmax(mx_err, part[4 * i + 1]);
    lo = fmin(lo, part[4 * i + 2]);
    hi = fmax(hi, part[4 * i + 3]);
  }
  sse = wg_sum<kQT>(sse, red);
  mx_err = wg_max<kQT>(mx_err, red);
  lo = wg_min<kQT>(lo, red);
  hi = wg_max<kQT>(hi, red);
  if (threadIdx.x == 0) {
    out[0] = sse;
    out[1] = mx_err;
    out[2] = lo;
    out[3] = hi;
  }
}

// wave-wide sum in a fixed order (tree toward lane 0), broadcast from lane 0
__device__ __forceinline__ double wave_sum(double v)
{
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return __shfl(v, 0, 64);
}

// One wave per window (windows in row-major order of their origins): the two
// means, then the centred second moments, then the window's SSIM.
template <typename T>
__global__ void __launch_bounds__(kQT) ssim_kernel(const T* __restrict__ x, const T* __restrict__ xr,
                                                   SsimGeom g, double* __restrict__ wout)
{
  const int lane = threadIdx.x & 63;
  const uint64_t wave = ((uint64_t)blockIdx.x * kQT + threadIdx.x) >> 6;
  const uint64_t nwave = ((uint64_t)gridDim.x * kQT) >> 6;
  const double inv = 1.0 / (double)g.cells;
  for (uint64_t wi = wave; wi < g.windows; wi += nwave) {
    // window origin
    uint64_t r = wi;
    int64_t o[4];
    for (int d = 3; d >= 0; d--) {
      const uint64_t q = r / g.nw[d];
      o[d] = (int64_t)(r - q * g.nw[d]) * g.s[d];
      r = q;
    }
    const int64_t base = o[0] * g.st[0] + o[1] * g.st[1] + o[2] * g.st[2] + o[3];
    auto addr = [&](uint32_t c) {
      // cell c of the window, row-major over the window sides
      uint32_t t = c;
      int64_t a = base;
      for (int d = 3; d >= 1; d--) {
        const uint32_t q = t / (uint32_t)g.s[d];
        a += (int64_t)(t - q * (uint32_t)g.s[d]) * g.st[d];
        t = q;
      }
      return a + (int64_t)t * g.st[0];
    };
    double sx = 0.0, sy = 0.0;
    for (uint32_t c = lane; c < g.cells; c += 64) {
      const int64_t a = addr(c);
      sx += (double)x[a];
      sy += (double)xr[a];
    }
    const double mx = wave_sum(sx) * inv, my = wave_sum(sy) * inv;
    double vxx = 0.0, vyy = 0.0, vxy = 0.0;
    for (uint32_t c = lane; c < g.cells; c += 64) {
      const int64_t a = addr(c);
      const double dx = (double)x[a] - mx, dy = (double)xr[a] - my;
      vxx += dx * dx;
      vyy += dy * dy;
      vxy += dx * dy;
    }
    const double sxx = wave_sum(vxx) * inv, syy = wave_sum(vyy) * inv, sxy = wave_sum(vxy) * inv;
    if (lane == 0)
      wout[wi] = ((2.0 * mx * my + g.c1) * (2.0 * sxy + g.c2)) /
                 ((mx * mx + my * my + g.c1) * (sxx + syy + g.c2));
  }
}

// per work-group sums of v[g * per, (g + 1) * per)
__global__ void __launch_bounds__(kQT) vsum_kernel(const double* __restrict__ v, uint64_t n,
                                                   uint64_t per, double* __restrict__ part)
{
  __shared__ double red[kQT];
  const uint64_t b = (uint64_t)blockIdx.x * per;
  const uint64_t e = b + per < n ? b + per : n;
  double s = 0.0;
  for (uint64_t i = b + threadIdx.x; i < e; i += kQT) s += v[i];
  s = wg_sum<kQT>(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kQT) vsum_final_kernel(const double* __restrict__ part, uint32_t np,
                                                         double* __restrict__ out)
{
  __shared__ double red[kQT];
  double s = 0.0;
  for (uint32_t i = threadIdx.x; i < np; i += kQT) s += part[i];
  s = wg_sum<kQT>(s, red);
  if (threadIdx.x == 0) out[0] = s;
}

}  // namespace

QGrid quality_grid(uint64_t n)
{
  // about 16 points per thread, at most kQMaxParts work-groups
  QGrid q;
  uint64_t parts = (n + (uint64_t)kQT * 16 - 1) / ((uint64_t)kQT * 16);
  if (parts < 1) parts = 1;
  if (parts > kQMaxParts) parts = kQMaxParts;
  q.per = (n + parts - 1) / parts;
  q.parts = (uint32_t)((n + q.per - 1) / q.per);
  if (q.parts < 1) q.parts = 1;
  return q;
}

template <typename T>
hipError_t launch_quality_sums(const T* x, const T* xr, uint64_t n, double* d_part, double* d_out,
                               hipStream_t st)
{
  const QGrid q = quality_grid(n);
  hipLaunchKernelGGL((qsum_kernel<T>), dim3(q.parts), dim3(kQT), 0, st, x, xr, n, q.per, d_part);
  hipLaunchKernelGGL(qsum_final_kernel, dim3(1), dim3(kQT), 0, st, d_part, q.parts, d_out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ssim(const T* x, const T* xr, const SsimGeom& g, double* d_win, double* d_part,
                       double* d_out, hipStream_t st)
{
  uint64_t wg = (g.windows + 3) / 4;  // four waves (windows) per work-group
  if (wg > (1u << 20)) wg = 1u << 20;
  if (wg < 1) wg = 1;
  hipLaunchKernelGGL((ssim_kernel<T>), dim3((unsigned)wg), dim3(kQT), 0, st, x, xr, g, d_win);
  const QGrid q = quality_grid(g.windows);
  hipLaunchKernelGGL(vsum_kernel, dim3(q.parts), dim3(kQT), 0, st, d_win, g.windows, q.per, d_part);
  hipLaunchKernelGGL(vsum_final_kernel, dim3(1), dim3(kQT), 0, st, d_part, q.parts, d_out);
  return hipGetLastError();
}

#define QINST(T)                                                                              \
  template hipError_t launch_quality_sums<T>(const T*, const T*, uint64_t, double*, double*,     \
                                             hipStream_t);                                       \
  template hipError_t launch_ssim<T>(const T*, const T*, const SsimGeom&, double*, double*,       \
                                     double*, hipStream_t);
QINST(float)
QINST(double)
QINST(uint8_t)
QINST(uint16_t)
QINST(int16_t)
QINST(int32_t)

}  // namespace hpez
