// quality.cpp -- the quality functions M of Sec. 3.1, Eq. (1) on the device
// (hpez_quality_eval) and the search for the largest error bound whose
// compression meets a quality requirement M >= m0 (hpez_fit_eb).
//
// Definitions (the paper names PSNR and SSIM without restating them; these
// are the usual ones):
//   value range L = max(X) - min(X); MSE = mean((x - x')^2);
//   PSNR = 20 log10(L) - 10 log10(MSE) (+inf for MSE = 0, -inf for L = 0 < MSE);
//   SSIM = mean over windows of ((2 mx my + C1)(2 sxy + C2)) /
//          ((mx^2 + my^2 + C1)(sx^2 + sy^2 + C2)), C1 = (0.01 L)^2,
//          C2 = (0.03 L)^2 (L = 1 for a constant field), population moments;
//          windows of side w along every dim of size > 1 (a shorter dim is one
//          window wide), without overlap from the origin, partial windows at
//          the far end left out.
#include <cmath>
#include <cstring>
#include <limits>

#include "hpez_host.h"
#include "hpez_internal.h"
#include "quality_dev.h"

namespace hpez {
namespace {

#define QCK(x)                                   \
  do {                                           \
    if ((x) != hipSuccess) return HPEZ_EDEVICE; \
  } while (0)

int check_shape(const hpez_field_desc* d)
{
  if (!d || d->dtype > HPEZ_I32 || d->ndims < 1 || d->ndims > 4) return HPEZ_EINVAL;
  uint64_t n = 1;
  for (int i = 0; i < d->ndims; i++) {
    if (d->dims[i] < 1 || d->dims[i] >= (1ull << 32)) return HPEZ_EINVAL;
    n *= d->dims[i];
    if (n >= (1ull << 32)) return HPEZ_EINVAL;
  }
  return HPEZ_OK;
}

uint64_t npoints(const hpez_field_desc* d)
{
  uint64_t n = 1;
  for (int i = 0; i < d->ndims; i++) n *= d->dims[i];
  return n;
}

SsimGeom ssim_geom(const hpez_field_desc* d, uint32_t w)
{
  SsimGeom g;
  std::memset(&g, 0, sizeof g);
  int64_t n[4] = {1, 1, 1, 1};
  for (int i = 0; i < d->ndims; i++) n[i] = (int64_t)d->dims[i];
  g.st[3] = 1;
  for (int i = 2; i >= 0; i--) g.st[i] = g.st[i + 1] * n[i + 1];
  g.windows = 1;
  uint64_t cells = 1;
  for (int i = 0; i < 4; i++) {
    if (n[i] <= 1) {
      g.s[i] = 1;
      g.nw[i] = 1;
    } else if (n[i] < (int64_t)w) {
      g.s[i] = n[i];
      g.nw[i] = 1;
    } else {
      g.s[i] = w;
      g.nw[i] = (uint64_t)(n[i] / w);
    }
    g.windows *= g.nw[i];
    cells *= (uint64_t)g.s[i];
  }
  g.cells = (uint32_t)cells;
  return g;
}

template <typename T>
int eval_t(hpez_ctx* ctx, const hpez_field_desc* d, const T* x, const T* xr, uint32_t w,
           hpez_quality* q, hipStream_t st)
{
  const uint64_t N = npoints(d);
  const SsimGeom g0 = ssim_geom(d, w);
  const size_t part_b = (size_t)4 * kQMaxParts * 8, out_b = 64;
  const size_t bytes = part_b + out_b + ((size_t)g0.windows * 8 + 255) / 256 * 256;
  int rc = HPEZ_OK;
  uint8_t* ws = (uint8_t*)ctx_ws(ctx, bytes, &rc);
  if (rc) return rc;
  uint8_t* pin = ctx_pin(ctx, 64, &rc);
  if (rc) return rc;
  double* d_part = (double*)ws;
  double* d_out = (double*)(ws + part_b);
  double* d_win = (double*)(ws + part_b + out_b);
  double* h = (double*)pin;
  QCK(launch_quality_sums<T>(x, xr, N, d_part, d_out, st));
  QCK(hipMemcpyAsync(h, d_out, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
  QCK(hipStreamSynchronize(st));
  const double sse = h[0], maxerr = h[1], lo = h[2], hi = h[3];
  if (!std::isfinite(sse) || !std::isfinite(lo) || !std::isfinite(hi)) return HPEZ_EINVAL;
  const double L = hi - lo;
  const double Ls = L == 0.0 ? 1.0 : L;
  SsimGeom g = g0;
  g.c1 = (0.01 * Ls) * (0.01 * Ls);
  g.c2 = (0.03 * Ls) * (0.03 * Ls);
  QCK(launch_ssim<T>(x, xr, g, d_win, d_part, d_out + 4, st));
  QCK(hipMemcpyAsync(h + 4, d_out + 4, sizeof(double), hipMemcpyDeviceToHost, st));
  QCK(hipStreamSynchronize(st));
  q->n = N;
  q->n_windows = g.windows;
  q->value_range = L;
  q->max_abs_err = maxerr;
  q->mse = sse / (double)N;
  if (q->mse == 0.0) q->psnr = std::numeric_limits<double>::infinity();
  else if (L == 0.0) q->psnr = -std::numeric_limits<double>::infinity();
  else q->psnr = 20.0 * std::log10(L) - 10.0 * std::log10(q->mse);
  q->ssim = h[4] / (double)g.windows;
  return HPEZ_OK;
}

// ---- the bound search: grid e_k = L 2^(k / G), G steps per octave
double grid_eb(double L, int64_t k, int G) { return L * std::pow(2.0, (double)k / (double)G); }

int64_t round_half_up(double v) { return (int64_t)std::floor(v + 0.5); }

// first index: PSNR by the uniform-quantizer model (MSE = e^2 / 3), SSIM at
// e / L = 10^-3
int64_t initial_k(int metric, double target, int G)
{
  const double r =
      metric == HPEZ_METRIC_PSNR ? std::sqrt(3.0) * std::pow(10.0, -target / 20.0) : 1e-3;
  return round_half_up((double)G * std::log2(r));
}

// steps suggested by a measured metric m (PSNR: 20 dB per decade of e; SSIM:
// deficit proportional to e^2), at least one step away from a met target (up)
// or a missed one (down), at most four octaves
int64_t model_step(int metric, double target, double m, int G)
{
  int64_t dk;
  if (metric == HPEZ_METRIC_PSNR)
    dk = std::isinf(m) ? 4 * (int64_t)G
                       : round_half_up((double)G * (m - target) / 20.0 * std::log2(10.0));
  else
    dk = m >= 1.0 ? 4 * (int64_t)G
                  : round_half_up((double)G * std::log2((1.0 - target) / (1.0 - m)) / 2.0);
  if (m >= target) return std::min<int64_t>(4 * (int64_t)G, std::max<int64_t>(1, dk));
  return std::max<int64_t>(-4 * (int64_t)G, std::min<int64_t>(-1, dk));
}

}  // namespace
}  // namespace hpez

using namespace hpez;

extern "C" {

int hpez_quality_eval(hpez_ctx* ctx, const hpez_field_desc* desc, const void* d_x, const void* d_xr,
                      uint32_t ssim_window, hpez_quality* out, hipStream_t stream)
{
  if (!ctx || !d_x || !d_xr || !out || check_shape(desc)) return HPEZ_EINVAL;
  const uint32_t w = ssim_window ? ssim_window : 8;
  if (w > 64) return HPEZ_EINVAL;
  const SsimGeom g = ssim_geom(desc, w);
  if (g.cells > (1u << 24)) return HPEZ_EINVAL;
  DeviceGuard dg(ctx_device(ctx));
  std::memset(out, 0, sizeof *out);
  switch (desc->dtype) {
    case HPEZ_F32:
      return eval_t<float>(ctx, desc, (const float*)d_x, (const float*)d_xr, w, out, stream);
    case HPEZ_F64:
      return eval_t<double>(ctx, desc, (const double*)d_x, (const double*)d_xr, w, out, stream);
    case HPEZ_U8:
      return eval_t<uint8_t>(ctx, desc, (const uint8_t*)d_x, (const uint8_t*)d_xr, w, out, stream);
    case HPEZ_U16:
      return eval_t<uint16_t>(ctx, desc, (const uint16_t*)d_x, (const uint16_t*)d_xr, w, out,
                              stream);
    case HPEZ_I16:
      return eval_t<int16_t>(ctx, desc, (const int16_t*)d_x, (const int16_t*)d_xr, w, out, stream);
    default:
      return eval_t<int32_t>(ctx, desc, (const int32_t*)d_x, (const int32_t*)d_xr, w, out, stream);
  }
}

int hpez_fit_eb(hpez_ctx* ctx, const hpez_field_desc* desc, const void* d_in,
                const hpez_config* cfg, const hpez_fit_opts* opts, hpez_fit_result* res,
                hipStream_t stream)
{
  if (!ctx || !d_in || !cfg || !opts || !res || check_shape(desc)) return HPEZ_EINVAL;
  if (opts->metric != HPEZ_METRIC_PSNR && opts->metric != HPEZ_METRIC_SSIM) return HPEZ_EINVAL;
  if (!std::isfinite(opts->target)) return HPEZ_EINVAL;
  if (opts->metric == HPEZ_METRIC_SSIM && !(opts->target < 1.0)) return HPEZ_EINVAL;
  const int G = opts->steps_per_octave ? (int)opts->steps_per_octave : 64;
  const int max_iter = opts->max_iter ? (int)opts->max_iter : 12;
  if (G > 1024 || max_iter > 64) return HPEZ_EINVAL;
  const uint32_t w = opts->ssim_window ? opts->ssim_window : 8;
  std::memset(res, 0, sizeof *res);
  DeviceGuard dg(ctx_device(ctx));

  // the value range, from the metrics of the field against itself
  hpez_quality self;
  int rc = hpez_quality_eval(ctx, desc, d_in, d_in, w, &self, stream);
  if (rc) return rc;
  const double L = self.value_range;
  res->e_hi = std::numeric_limits<double>::infinity();
  if (L == 0.0) {
    // a constant field is reproduced exactly at any bound
    res->e = 0.0;
    res->quality = self;
    return HPEZ_OK;
  }
  hpez_field_desc dd = *desc;
  dd.eb_mode = HPEZ_ABS;
  dd.eb = L;
  uint64_t cap = 0;
  rc = hpez_compress_bound(&dd, cfg, &cap);
  if (rc) return rc;
  const uint64_t N = npoints(desc), s = dtype_size(desc->dtype);
  void* d_z = nullptr;
  void* d_xr = nullptr;
  if (hipMalloc(&d_z, cap) != hipSuccess) return HPEZ_ENOMEM;
  if (hipMalloc(&d_xr, N * s) != hipSuccess) {
    (void)hipFree(d_z);
    return HPEZ_ENOMEM;
  }
  int64_t k = initial_k(opts->metric, opts->target, G);
  bool have_lo = false, have_hi = false;
  int64_t k_lo = 0, k_hi = 0;
  int it = 0;
  while (it < max_iter) {
    dd.eb = grid_eb(L, k, G);
    uint64_t size = 0;
    rc = hpez_compress(ctx, &dd, d_in, cfg, d_z, cap, &size, stream);
    if (!rc) rc = hpez_decompress(ctx, d_z, size, d_xr, N * s, stream);
    hpez_quality q;
    if (!rc) rc = hpez_quality_eval(ctx, desc, d_in, d_xr, w, &q, stream);
    if (rc) break;
    it++;
    const double m = opts->metric == HPEZ_METRIC_PSNR ? q.psnr : q.ssim;
    if (m >= opts->target) {
      if (!have_lo || k > k_lo) {
        k_lo = k;
        have_lo = true;
        res->quality = q;
        res->bytes = size;
      }
    } else if (!have_hi || k < k_hi) {
      k_hi = k;
      have_hi = true;
    }
    if (have_lo && have_hi) {
      if (k_hi - k_lo <= 1) break;
      k = k_lo + (k_hi - k_lo) / 2;
    } else {
      k += model_step(opts->metric, opts->target, m, G);
    }
  }
  (void)hipFree(d_z);
  (void)hipFree(d_xr);
  if (rc) return rc;
  res->iterations = (uint32_t)it;
  res->e = have_lo ? grid_eb(L, k_lo, G) : 0.0;
  res->e_hi = have_hi ? grid_eb(L, k_hi, G) : std::numeric_limits<double>::infinity();
  return HPEZ_OK;
}

}  // extern "C"
