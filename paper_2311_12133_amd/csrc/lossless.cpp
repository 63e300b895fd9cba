// lossless.cpp -- the lossless stage after Huffman coding (Sec. 4, step 5):
// hpez_lossless_encode / hpez_lossless_decode.
//
// The paper passes the Huffman-coded stream through a general-purpose
// lossless compressor; what such a compressor finds there is mostly runs of
// zero bytes (the one-bit codeword 0 of the most frequent quantization code).
// This stage codes the zero runs as tokens (lossless_dev.h) and Huffman-codes
// the tokens with the quantization codes' own encoder and decoder, so every
// step is data-parallel on the device; the codebook is built on the host from
// the token histogram, as for the codes.  The result is stored instead when it
// is not smaller.
//
// Container (little-endian):
//    0 u32 magic "HPZL"  4 u16 version 1  6 u16 mode (0 stored, 1 coded)
//    8 u64 n  16 u64 n_tokens  24 u64 payload_bits  32 u32 chunk (1024)
//   36 u32 sym_min  40 u32 sym_max  44 u32 kRunMax
//   48 mode 0: the n bytes; mode 1: code lengths u8[sym_max - sym_min + 1],
//      padded to 8; chunk bit counts u16[ceil(n_tokens / chunk)], padded to 8;
//      payload u32[ceil(payload_bits / 32)].
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "codec_dev.h"
#include "hpez_host.h"
#include "lossless_dev.h"

namespace hpez {
namespace {

#define LLCK(x)                                 \
  do {                                          \
    if ((x) != hipSuccess) return HPEZ_EDEVICE; \
  } while (0)

constexpr uint32_t kLLMagic = 0x4C5A5048u;
constexpr uint64_t kLLHdr = 48;
constexpr uint32_t kLLChunk = 1024;

uint64_t al8(uint64_t v) { return (v + 7) & ~7ull; }
size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

struct LLHeader {
  uint16_t mode = 0;
  uint64_t n = 0, ntok = 0, bits = 0;
  uint32_t smin = 0, smax = 0;
  uint64_t off_len = kLLHdr, off_chunks = 0, off_payload = 0, nch = 0, total = 0;
};

void ll_layout(LLHeader& h)
{
  if (h.mode == 0) {
    h.total = kLLHdr + h.n;
    return;
  }
  h.off_len = kLLHdr;
  h.off_chunks = al8(h.off_len + h.smax - h.smin + 1);
  h.nch = (h.ntok + kLLChunk - 1) / kLLChunk;
  h.off_payload = al8(h.off_chunks + 2 * h.nch);
  h.total = h.off_payload + 4 * ((h.bits + 31) / 32);
}

void ll_write_header(uint8_t* p, const LLHeader& h)
{
  std::memset(p, 0, kLLHdr);
  const uint16_t ver = 1;
  const uint32_t chunk = kLLChunk, rmax = kRunMax;
  std::memcpy(p, &kLLMagic, 4);
  std::memcpy(p + 4, &ver, 2);
  std::memcpy(p + 6, &h.mode, 2);
  std::memcpy(p + 8, &h.n, 8);
  std::memcpy(p + 16, &h.ntok, 8);
  std::memcpy(p + 24, &h.bits, 8);
  std::memcpy(p + 32, &chunk, 4);
  std::memcpy(p + 36, &h.smin, 4);
  std::memcpy(p + 40, &h.smax, 4);
  std::memcpy(p + 44, &rmax, 4);
}

int ll_read_header(const uint8_t* p, uint64_t in_size, LLHeader* h)
{
  if (in_size < kLLHdr) return HPEZ_ECORRUPT;
  uint32_t magic, chunk, rmax;
  uint16_t ver;
  std::memcpy(&magic, p, 4);
  std::memcpy(&ver, p + 4, 2);
  std::memcpy(&h->mode, p + 6, 2);
  std::memcpy(&h->n, p + 8, 8);
  std::memcpy(&h->ntok, p + 16, 8);
  std::memcpy(&h->bits, p + 24, 8);
  std::memcpy(&chunk, p + 32, 4);
  std::memcpy(&h->smin, p + 36, 4);
  std::memcpy(&h->smax, p + 40, 4);
  std::memcpy(&rmax, p + 44, 4);
  if (magic != kLLMagic || ver != 1 || h->mode > 1 || chunk != kLLChunk || rmax != kRunMax)
    return HPEZ_ECORRUPT;
  if (h->mode == 1) {
    if (!(h->smin >= 1 && h->smin <= h->smax && h->smax < kTokSyms) || h->ntok == 0 ||
        h->ntok > h->n || h->bits < h->ntok || h->bits > h->ntok * (uint64_t)kLmax)
      return HPEZ_ECORRUPT;
  }
  ll_layout(*h);
  return h->total == in_size ? HPEZ_OK : HPEZ_ECORRUPT;
}

struct Bump {
  uint8_t* p;
  template <typename T>
  T* take(size_t count)
  {
    T* r = reinterpret_cast<T*>(p);
    p += al256(count * sizeof(T));
    return r;
  }
};

}  // namespace
}  // namespace hpez

using namespace hpez;

extern "C" {

int hpez_lossless_bound(uint64_t n, uint64_t* out_bytes)
{
  if (!out_bytes) return HPEZ_EINVAL;
  *out_bytes = kLLHdr + n;
  return HPEZ_OK;
}

int hpez_lossless_encode(hpez_ctx* ctx, const void* d_in, uint64_t n, void* d_out,
                         uint64_t out_cap, uint64_t* out_size, hipStream_t st)
{
  if (!ctx || !d_out || !out_size || (n && !d_in)) return HPEZ_EINVAL;
  if (n >= 0xFFFFFFFFull) return HPEZ_EUNSUPPORTED;  // 32-bit byte positions
  if (out_cap < kLLHdr + n) return HPEZ_ENOSPC;
  DeviceGuard dg(ctx_device(ctx));
  const uint8_t* in = (const uint8_t*)d_in;
  uint8_t* out = (uint8_t*)d_out;
  int rc;
  // pinned: header, histogram, lengths, codewords, packed table
  const size_t pin_bytes = 64 + kTokSyms * 4 + 16 + al256(kTokSyms) + kTokSyms * 4 + kTokSyms * 4 +
                           al256(kTokSyms) + 1024;
  uint8_t* pin = ctx_pin(ctx, pin_bytes, &rc);
  if (rc) return rc;
  uint8_t* h_hdr = pin;
  uint32_t* h_hist = reinterpret_cast<uint32_t*>(pin + 64);
  uint64_t* h_ntok = reinterpret_cast<uint64_t*>(pin + 64 + kTokSyms * 4);
  uint8_t* h_len = pin + 64 + kTokSyms * 4 + 16;
  uint32_t* h_cw = reinterpret_cast<uint32_t*>(h_len + al256(kTokSyms));
  uint32_t* h_tab = h_cw + kTokSyms;
  LLHeader h;
  h.n = n;
  if (n == 0) {
    ll_layout(h);
    ll_write_header(h_hdr, h);
    LLCK(hipMemcpyAsync(out, h_hdr, kLLHdr, hipMemcpyHostToDevice, st));
    LLCK(hipStreamSynchronize(st));
    *out_size = h.total;
    return HPEZ_OK;
  }
  const uint64_t ntile = (n + kLLTile - 1) / kLLTile;
  const uint64_t nmax_ch = (n + kLLChunk - 1) / kLLChunk;
  const size_t need = al256((ntile + 1) * 4) + al256((ntile + 1) * 8) + al256((n + 1) * 4) +
                      al256((n + 1) * 4) + al256((n + 2) * 8) + al256((n + 1) * 2) +
                      al256(kTokSyms * 4) + al256(kTokSyms) + al256(kTokSyms * 4) +
                      al256((nmax_ch + 1) * 8) + al256(((n + 1) / 1024 + 2) * 8) + 2 * 256;
  Bump bw{(uint8_t*)ctx_ws(ctx, need, &rc)};
  if (rc) return rc;
  uint32_t* cnt = bw.take<uint32_t>(ntile + 1);
  uint64_t* toff_tile = bw.take<uint64_t>(ntile + 1);
  uint32_t* pos = bw.take<uint32_t>(n + 1);
  uint32_t* tcnt = bw.take<uint32_t>(n + 1);
  uint64_t* toff = bw.take<uint64_t>(n + 2);
  uint16_t* tok = bw.take<uint16_t>(n + 1);
  uint32_t* hist = bw.take<uint32_t>(kTokSyms);
  uint8_t* dlen = bw.take<uint8_t>(kTokSyms);
  uint32_t* dcw = bw.take<uint32_t>(kTokSyms);
  uint64_t* flags = bw.take<uint64_t>(nmax_ch + 1);
  uint64_t* tmp1 = bw.take<uint64_t>((n + 1) / 1024 + 2);
  uint64_t* scal = bw.take<uint64_t>(4);  // nnz, n_tokens
  uint32_t* ticket = bw.take<uint32_t>(4);
  // tokens and their histogram
  {
    hipEvent_t ev = ctx_span_begin(ctx, st, "lossless_tokens");
    LLCK(hipMemsetAsync(hist, 0, kTokSyms * 4, st));
    LLCK(launch_ll_count(in, n, cnt, st));
    LLCK(launch_scan_u32_to_u64(cnt, ntile, toff_tile, &scal[0], tmp1, st));
    LLCK(launch_ll_compact(in, n, toff_tile, pos, st));
    LLCK(launch_ll_tokcount(pos, &scal[0], n, tcnt, st));
    LLCK(launch_scan_u32_to_u64(tcnt, n + 1, toff, &scal[1], tmp1, st));
    LLCK(launch_ll_tokens(in, pos, &scal[0], n, toff, tok, hist, st));
    ctx_span_end(ctx, ev, "lossless_tokens", n * 2, st);
  }
  LLCK(hipMemcpyAsync(h_hist, hist, kTokSyms * 4, hipMemcpyDeviceToHost, st));
  LLCK(hipMemcpyAsync(h_ntok, &scal[1], 8, hipMemcpyDeviceToHost, st));
  LLCK(hipStreamSynchronize(st));
  // codebook and layout
  h.ntok = *h_ntok;
  rc = huffman_lengths(h_hist, kTokSyms, h_len);
  if (rc) return rc;
  uint32_t smin = kTokSyms, smax = 0;
  uint64_t bits = 0;
  for (uint32_t s = 0; s < kTokSyms; s++) {
    if (!h_len[s]) continue;
    smin = s < smin ? s : smin;
    smax = s;
    bits += (uint64_t)h_hist[s] * h_len[s];
  }
  h.mode = 1;
  h.bits = bits;
  h.smin = smin;
  h.smax = smax;
  ll_layout(h);
  if (h.ntok == 0 || smin > smax || h.total >= kLLHdr + n) {
    // stored
    LLHeader s;
    s.n = n;
    ll_layout(s);
    ll_write_header(h_hdr, s);
    LLCK(hipMemcpyAsync(out, h_hdr, kLLHdr, hipMemcpyHostToDevice, st));
    LLCK(hipMemcpyAsync(out + kLLHdr, in, n, hipMemcpyDeviceToDevice, st));
    LLCK(hipStreamSynchronize(st));
    *out_size = s.total;
    return HPEZ_OK;
  }
  canonical_codes_range(h_len, smin, smax + 1, h_cw);
  // header, code lengths and padding in one upload
  uint8_t* img = reinterpret_cast<uint8_t*>(h_tab + kTokSyms);
  const uint64_t nl = smax - smin + 1;
  std::memset(img, 0, h.off_chunks);
  ll_write_header(img, h);
  std::memcpy(img + kLLHdr, h_len + smin, nl);
  LLCK(hipMemsetAsync(out + h.off_chunks, 0, h.total - h.off_chunks, st));
  LLCK(hipMemcpyAsync(out, img, h.off_chunks, hipMemcpyHostToDevice, st));
  // the encoder's full tables when its packed table cannot hold every codeword
  uint32_t nlong = 0;
  for (uint32_t s = smin; s <= smax; s++) nlong += h_len[s] > 26;
  if (((nl + 1) & ~1ull) + 2ull * nlong > kTokSyms) {
    for (uint32_t s = 0; s < kTokSyms; s++)
      if (!h_len[s]) h_cw[s] = 0;
    LLCK(hipMemcpyAsync(dlen, h_len, kTokSyms, hipMemcpyHostToDevice, st));
    LLCK(hipMemcpyAsync(dcw, h_cw, kTokSyms * 4, hipMemcpyHostToDevice, st));
  }
  rc = encode_payload(ctx, tok, h.ntok, kLLChunk, h_len, h_cw, smin, smax, dlen, dcw, hist,
                      kTokSyms, flags, ticket, h_tab, reinterpret_cast<uint32_t*>(out + h.off_payload),
                      reinterpret_cast<uint16_t*>(out + h.off_chunks), st);
  if (rc) {
    ctx_drain(ctx, st);
    return rc;
  }
  LLCK(hipStreamSynchronize(st));
  ctx_prof_collect(ctx);
  *out_size = h.total;
  return HPEZ_OK;
}

int hpez_lossless_decode(hpez_ctx* ctx, const void* d_in, uint64_t in_size, void* d_out,
                         uint64_t out_cap, uint64_t* out_size, hipStream_t st)
{
  if (!ctx || !d_in || !out_size) return HPEZ_EINVAL;
  DeviceGuard dg(ctx_device(ctx));
  const uint8_t* in = (const uint8_t*)d_in;
  uint8_t* out = (uint8_t*)d_out;
  int rc;
  // pinned: prefix (header + lengths), table image, status read-back
  const uint64_t pre = kLLHdr + kTokSyms;
  const size_t img_bytes = 16 + (4u << kLutBits) + (size_t)kDecSub * 4 + kTokSyms * 2 + 64;
  uint8_t* pin = ctx_pin(ctx, al256(pre) + al256(img_bytes) + 64 + kTokSyms * 2, &rc);
  if (rc) return rc;
  uint8_t* h_pre = pin;
  uint8_t* h_img = pin + al256(pre);
  int* h_status = reinterpret_cast<int*>(h_img + al256(img_bytes));
  uint64_t* h_tot = reinterpret_cast<uint64_t*>(h_status + 4);
  uint16_t* h_sorted = reinterpret_cast<uint16_t*>(h_tot + 2);
  if (in_size < kLLHdr) return HPEZ_ECORRUPT;
  LLCK(hipMemcpyAsync(h_pre, in, in_size < pre ? in_size : pre, hipMemcpyDeviceToHost, st));
  LLCK(hipStreamSynchronize(st));
  LLHeader h;
  rc = ll_read_header(h_pre, in_size, &h);
  if (rc) return rc;
  *out_size = h.n;
  if (out_cap < h.n) return HPEZ_ENOSPC;
  if (h.n && !out) return HPEZ_EINVAL;
  if (h.mode == 0) {
    if (h.n) LLCK(hipMemcpyAsync(out, in + kLLHdr, h.n, hipMemcpyDeviceToDevice, st));
    return HPEZ_OK;
  }
  // code lengths: a complete prefix code (Kraft sum one, or a single symbol)
  uint8_t len[kTokSyms];
  std::memset(len, 0, sizeof len);
  std::memcpy(len + h.smin, h_pre + kLLHdr, h.smax - h.smin + 1);
  uint64_t kraft = 0, used = 0;
  for (uint32_t s = h.smin; s <= h.smax; s++) {
    if (!len[s]) continue;
    if (len[s] > kLmax) return HPEZ_ECORRUPT;
    kraft += 1ull << (kLmax - len[s]);
    used++;
  }
  if (!(kraft == (1ull << kLmax) || (used == 1 && kraft == (1ull << (kLmax - 1)))))
    return HPEZ_ECORRUPT;
  // decode tables (the quantization codes' decoder), one upload: status and
  // ticket, first-level table, second-level tables, sorted symbols; the tile
  // flags after them are cleared on the device
  DecodeArgs da;
  std::memset(&da, 0, sizeof da);
  da.n = h.ntok;
  da.nch = h.nch;
  da.nbits = h.bits;
  da.chunk = kLLChunk;
  uint32_t* lut = reinterpret_cast<uint32_t*>(h_img + 16);
  uint32_t* sub = lut + (1u << kLutBits);
  decode_tables_range(len, h.smin, h.smax + 1, lut, h_sorted, da.lim, da.base);
  uint32_t nshort = 0;
  for (uint32_t s = h.smin; s <= h.smax; s++) nshort += len[s] && len[s] <= kLutBits;
  da.long_first = nshort;
  da.n_long = (uint32_t)used - nshort;
  da.n_sub = da.n_long ? decode_subtables(len, h.smin, h.smax + 1, lut, sub, kDecSub) : 0;
  const uint64_t so = 16 + (4ull << kLutBits) + (uint64_t)da.n_sub * 4;
  std::memcpy(h_img + so, h_sorted, used * 2);
  std::memset(h_img, 0, 16);
  const uint64_t fo = al8(so + used * 2);
  const uint64_t nfl = (h.nch + 255) / 256;
  const uint64_t tabs = fo + nfl * 8;
  const size_t need = al256(tabs) + al256((h.ntok + 1) * 2) + al256((h.nch + 1) * 4) +
                      al256((h.ntok + 1) * 4) + al256((h.ntok + 1) * 8) +
                      al256((h.ntok + 1) / 1024 + 2) * 8 + 256 * 4;
  Bump bw{(uint8_t*)ctx_ws(ctx, need, &rc)};
  if (rc) return rc;
  uint8_t* dtabs = bw.take<uint8_t>(tabs);
  uint16_t* tok = bw.take<uint16_t>(h.ntok + 1);
  uint32_t* czero = bw.take<uint32_t>(h.nch + 1);
  uint32_t* tlen = bw.take<uint32_t>(h.ntok + 1);
  uint64_t* off = bw.take<uint64_t>(h.ntok + 1);
  uint64_t* tmp = bw.take<uint64_t>((h.ntok + 1) / 1024 + 2);
  uint64_t* total = bw.take<uint64_t>(2);
  LLCK(hipMemcpyAsync(dtabs, h_img, fo, hipMemcpyHostToDevice, st));
  LLCK(hipMemsetAsync(dtabs + fo, 0, nfl * 8, st));
  int* status = reinterpret_cast<int*>(dtabs);
  {
    hipEvent_t ev = ctx_span_begin(ctx, st, "lossless_expand");
    LLCK(launch_decode2(da, reinterpret_cast<const uint32_t*>(in + h.off_payload),
                        reinterpret_cast<const uint16_t*>(in + h.off_chunks),
                        reinterpret_cast<uint64_t*>(dtabs + fo), reinterpret_cast<uint32_t*>(dtabs + 16),
                        reinterpret_cast<const uint16_t*>(dtabs + so),
                        reinterpret_cast<uint32_t*>(dtabs + 16 + (4ull << kLutBits)), tok, czero,
                        status, st));
    LLCK(launch_ll_toklen(tok, h.ntok, tlen, status, st));
    LLCK(launch_scan_u32_to_u64(tlen, h.ntok, off, total, tmp, st));
    LLCK(hipMemsetAsync(out, 0, h.n, st));
    LLCK(launch_ll_expand(tok, h.ntok, off, out, h.n, status, st));
    ctx_span_end(ctx, ev, "lossless_expand", h.n + (h.bits + 7) / 8, st);
  }
  LLCK(hipMemcpyAsync(h_status, status, 4, hipMemcpyDeviceToHost, st));
  LLCK(hipMemcpyAsync(h_tot, total, 8, hipMemcpyDeviceToHost, st));
  LLCK(hipStreamSynchronize(st));
  ctx_prof_collect(ctx);
  if (*h_status || *h_tot != h.n) return HPEZ_ECORRUPT;
  return HPEZ_OK;
}

}  // extern "C"
