// lorenzo.cpp -- host side of the Lorenzo alternative (Sec. 6.5): codes by
// dual-quantized first-order Lorenzo residuals, then the same histogram and
// Huffman stages as the interpolation predictor.  Residuals of magnitude >= R
// go to the outlier section (code 0); points whose rebuilt value misses the
// bound are listed in the patch sections.

#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "hpez_host.h"
#include "codec_dev.h"
#include "lorenzo_dev.h"

namespace hpez {

#define LCK(x)                                  \
  do {                                          \
    if ((x) != hipSuccess) return HPEZ_EDEVICE; \
  } while (0)

template <typename T>
int lorenzo_compress(hpez_ctx* ctx, const hpez_field_desc* d, const T* X, const hpez_config* c,
                     double e, uint8_t* out, uint64_t cap, uint64_t* out_size, hipStream_t st)
{
  const uint64_t N = points_of(d);
  const uint64_t s = sizeof(T);
  const uint32_t nsym = 2 * c->radius;
  const uint64_t nb = n_blocks(d, c);
  const uint64_t nch = (N + c->chunk - 1) / c->chunk;
  const Geom g = make_geom(d, -1);
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t ntile = (nch + 1023) / 1024 + 1;
  const size_t need = al(N * 2) + 3 * al((nch + 1) * 4) + 3 * al((nch + 1) * 8) +
                      3 * al(ntile * 8) + al(nsym * 4) + al(nsym) + al(nsym * 4) + al(64);
  int rc;
  uint8_t* base = (uint8_t*)ctx_ws(ctx, need, &rc);
  if (rc) return rc;
  uint8_t* pin = ctx_pin(ctx, nsym * 4 + nsym + kHdrBytes + 128 + nsym * 4, &rc);
  if (rc) return rc;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    uint8_t* p = base + off;
    off += al(bytes);
    return p;
  };
  uint16_t* code = (uint16_t*)take(N * 2);
  uint32_t* pcount = (uint32_t*)take((nch + 1) * 4);
  uint32_t* cbits = (uint32_t*)take((nch + 1) * 4);
  uint32_t* czero = (uint32_t*)take((nch + 1) * 4);
  uint64_t* poff = (uint64_t*)take((nch + 1) * 8);
  uint64_t* boff = (uint64_t*)take((nch + 1) * 8);
  uint64_t* zoff = (uint64_t*)take((nch + 1) * 8);
  uint64_t* t1 = (uint64_t*)take(ntile * 8);
  uint64_t* t2 = (uint64_t*)take(ntile * 8);
  uint64_t* t3 = (uint64_t*)take(ntile * 8);
  uint32_t* hist = (uint32_t*)take(nsym * 4);
  uint8_t* dlen = (uint8_t*)take(nsym);
  uint32_t* dcw = (uint32_t*)take(nsym * 4);
  int* bad = (int*)take(64);
  uint32_t* h_hist = (uint32_t*)pin;
  uint8_t* h_len = pin + nsym * 4;
  uint8_t* h_hdr = h_len + nsym;
  uint64_t* h_np = (uint64_t*)(h_hdr + kHdrBytes);
  int* h_bad = (int*)(h_np + 1);
  uint32_t* h_tab = (uint32_t*)(pin + (((size_t)nsym * 5 + kHdrBytes + 64 + 63) & ~(size_t)63));

  LorenzoArgs a;
  a.inv2e = 1.0 / (2.0 * e);
  a.twoe = 2.0 * e;
  a.e = e;
  a.R = c->radius;
  a.chunk = c->chunk;
  LCK(hipMemsetAsync(pcount, 0, (nch + 1) * 4, st));
  LCK(hipMemsetAsync(bad, 0, 4, st));
  hipEvent_t ev = ctx_span_begin(ctx, st, "lorenzo_codes");
  LCK(launch_lorenzo_codes<T>(X, g, N, a, code, pcount, bad, st));
  ctx_span_end(ctx, ev, "lorenzo_codes", N * (s + 2), st);
  LCK(hipMemsetAsync(hist, 0, (size_t)nsym * 4, st));
  LCK(launch_histogram(code, N, hist, nsym, c->radius, st));
  LCK(launch_scan_u32_to_u64(pcount, nch, poff, poff + nch, t1, st));
  LCK(hipMemcpyAsync(h_hist, hist, (size_t)nsym * 4, hipMemcpyDeviceToHost, st));
  LCK(hipMemcpyAsync(h_np, poff + nch, 8, hipMemcpyDeviceToHost, st));
  LCK(hipMemcpyAsync(h_bad, bad, 4, hipMemcpyDeviceToHost, st));
  LCK(hipStreamSynchronize(st));
  if (*h_bad) return HPEZ_EUNSUPPORTED;
  rc = huffman_lengths(h_hist, nsym, h_len);
  if (rc) return rc;
  std::vector<uint32_t> cw(nsym);
  canonical_codes(h_len, nsym, cw.data());
  Layout Lo;
  std::memset(&Lo, 0, sizeof Lo);
  Lo.predictor = 1;
  Lo.e = e;
  Lo.n_blocks = nb;
  Lo.sym_min = 1;
  Lo.sym_max = 0;
  uint64_t bits = 0;
  for (uint32_t k = 0; k < nsym; k++) bits += (uint64_t)h_hist[k] * h_len[k];
  for (uint32_t k = 0; k < nsym; k++)
    if (h_len[k]) { Lo.sym_min = k; break; }
  for (uint32_t k = nsym; k-- > 0;)
    if (h_len[k]) { Lo.sym_max = k; break; }
  Lo.n_outlier = h_hist[0];
  Lo.n_patch = *h_np;
  Lo.n_chunks = nch;
  Lo.payload_bits = bits;
  layout(&Lo, s);
  if (Lo.total > cap) return HPEZ_ENOSPC;
  write_header(h_hdr, d, c, Lo);
  LCK(hipMemcpyAsync(dlen, h_len, nsym, hipMemcpyHostToDevice, st));
  LCK(hipMemcpyAsync(dcw, cw.data(), (size_t)nsym * 4, hipMemcpyHostToDevice, st));
  LCK(hipMemsetAsync(out, 0, Lo.total, st));
  LCK(hipMemcpyAsync(out, h_hdr, kHdrBytes, hipMemcpyHostToDevice, st));
  if (nb) LCK(hipMemcpyAsync(out + Lo.off_blocks, c->block_cfg, nb, hipMemcpyHostToDevice, st));
  if (Lo.sym_max >= Lo.sym_min)
    LCK(hipMemcpyAsync(out + Lo.off_len, h_len + Lo.sym_min, Lo.sym_max - Lo.sym_min + 1,
                       hipMemcpyHostToDevice, st));
  LCK(launch_count_zeros(code, N, c->chunk, czero, zoff, t3, st));
  rc = encode_payload(ctx, code, N, c->chunk, h_len, cw.data(), Lo.sym_min, Lo.sym_max, dlen, dcw,
                      hist, nsym, boff, (uint32_t*)bad, h_tab, (uint32_t*)(out + Lo.off_payload),
                      (uint16_t*)(out + Lo.off_chunks), st);
  if (rc) return rc;
  LCK(launch_lorenzo_gather<T>(X, g, N, a, code, czero, zoff, pcount, poff,
                               (long long*)(out + Lo.off_outl), (uint64_t*)(out + Lo.off_pidx),
                               (T*)(out + Lo.off_pval), st));
  LCK(hipStreamSynchronize(st));
  ctx_prof_collect(ctx);
  *out_size = Lo.total;
  return HPEZ_OK;
}

template int lorenzo_compress<float>(hpez_ctx*, const hpez_field_desc*, const float*,
                                     const hpez_config*, double, uint8_t*, uint64_t, uint64_t*,
                                     hipStream_t);
template int lorenzo_compress<double>(hpez_ctx*, const hpez_field_desc*, const double*,
                                      const hpez_config*, double, uint8_t*, uint64_t, uint64_t*,
                                      hipStream_t);

}  // namespace hpez
