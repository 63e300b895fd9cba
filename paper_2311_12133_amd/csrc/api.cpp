// api.cpp -- host runtime and C ABI of the MI355X HPEZ library.
//
// Orchestrates the kernels of the compression pipeline (Sec. 4): error bound,
// level-wise interpolation with quantization (Sec. 5), histogram, Huffman
// codebook, encode; and the matching decompression.  Owns the stream format.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "hpez_internal.h"
#include "hpez_host.h"
#include "lorenzo_dev.h"
#include "block_dev.h"
#include "codec_dev.h"

using namespace hpez;

struct ProfRec {
  hipEvent_t a, b;
  const char* name;
  uint64_t bytes;
};

struct hpez_ctx {
  int device = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  uint8_t* pinned = nullptr;
  size_t pinned_bytes = 0;
  uint8_t* pin_tab = nullptr;  // staging of the block phase's work tables
  size_t pin_tab_bytes = 0;
  // kernel timing (hpez_profile_enable)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<ProfRec> pend;
  std::vector<hpez_kernel_stat> stats;

  hipEvent_t take_event()
  {
    if (ev_used == ev_pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ev_pool.push_back(e);
    }
    return ev_pool[ev_used++];
  }
};

namespace {

// Brackets a group of kernel launches with events while profiling is on.
struct Span {
  hpez_ctx* c;
  hipStream_t st;
  const char* name;
  uint64_t bytes;
  hipEvent_t a = nullptr;
  Span(hpez_ctx* c_, const char* name_, uint64_t bytes_, hipStream_t st_)
      : c(c_), st(st_), name(name_), bytes(bytes_)
  {
    if (c && c->prof) {
      a = c->take_event();
      if (a && hipEventRecord(a, st) != hipSuccess) a = nullptr;
    }
  }
  ~Span()
  {
    if (!a) return;
    hipEvent_t b = c->take_event();
    if (b && hipEventRecord(b, st) == hipSuccess) c->pend.push_back({a, b, name, bytes});
  }
};

// Fold finished spans into the per-name totals (call after a stream sync).
void prof_collect(hpez_ctx* c)
{
  for (const ProfRec& r : c->pend) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
    hpez_kernel_stat* s = nullptr;
    for (auto& x : c->stats)
      if (std::strncmp(x.name, r.name, sizeof x.name) == 0) s = &x;
    if (!s) {
      hpez_kernel_stat z;
      std::memset(&z, 0, sizeof z);
      std::strncpy(z.name, r.name, sizeof z.name - 1);
      c->stats.push_back(z);
      s = &c->stats.back();
    }
    s->launches++;
    s->bytes += r.bytes;
    s->total_ms += ms;
  }
  c->pend.clear();
  c->ev_used = 0;
}

}  // namespace

namespace hpez {

const char* err_text(int c)
{
  switch (c) {
    case HPEZ_OK: return "ok";
    case HPEZ_EINVAL: return "invalid argument";
    case HPEZ_ENOMEM: return "out of memory";
    case HPEZ_EDEVICE: return "HIP device error";
    case HPEZ_ECORRUPT: return "corrupt stream";
    case HPEZ_ENOSPC: return "output buffer too small";
    case HPEZ_EUNSUPPORTED: return "unsupported";
    default: return "unknown error";
  }
}

// ---------------------------------------------------------------------------
// validation and geometry

uint64_t points_of(const hpez_field_desc* d)
{
  uint64_t n = 1;
  for (int i = 0; i < d->ndims; i++) n *= d->dims[i];
  return n;
}

int check_desc(const hpez_field_desc* d)
{
  if (!d || d->dtype > 1 || d->ndims < 1 || d->ndims > 4 || d->eb_mode > 1) return HPEZ_EINVAL;
  if (!(d->eb > 0) || !std::isfinite(d->eb)) return HPEZ_EINVAL;
  uint64_t n = 1;
  for (int i = 0; i < d->ndims; i++) {
    if (d->dims[i] < 1 || d->dims[i] >= (1ull << 32)) return HPEZ_EINVAL;
    n *= d->dims[i];
    if (n >= (1ull << 32)) return HPEZ_EINVAL;
  }
  return HPEZ_OK;
}

static bool interp_ok(const hpez_interp& c, int ndims)
{
  if (c.kind > 2 || c.md > 1 || c.same_level > 1) return false;
  bool seen[4] = {false, false, false, false};
  for (int j = 0; j < ndims; j++) {
    if (c.order[j] >= ndims || seen[c.order[j]]) return false;
    seen[c.order[j]] = true;
  }
  return true;
}

int check_cfg(const hpez_field_desc* d, const hpez_config* c, bool need_blocks)
{
  if (!c) return HPEZ_EINVAL;
  if (c->predictor > 1 || c->anchor_log2 > 16 || c->block_log2 > 15) return HPEZ_EINVAL;
  if (c->radius < 1 || c->radius > 32768) return HPEZ_EINVAL;
  if (c->chunk < 64 || c->chunk > 1024 || (c->chunk & (c->chunk - 1))) return HPEZ_EINVAL;
  if (!(c->alpha >= 1.0) || !(c->beta >= 1.0)) return HPEZ_EINVAL;
  if (c->frozen_dim < -1 || c->frozen_dim >= d->ndims) return HPEZ_EINVAL;
  if (c->n_cand > 16) return HPEZ_EINVAL;
  for (int k = 0; k < 3; k++)
    for (int j = 0; j < 4; j++)
      if (!(c->md_w[k][j] > 0) || !std::isfinite(c->md_w[k][j])) return HPEZ_EINVAL;
  for (int i = 0; i < 16; i++)
    if (!interp_ok(c->level[i], d->ndims)) return HPEZ_EINVAL;
  for (uint32_t i = 0; i < c->n_cand; i++)
    if (!interp_ok(c->cand[i], d->ndims)) return HPEZ_EINVAL;
  if (c->block_log2 && need_blocks) {
    if (c->n_cand < 1 || !c->block_cfg) return HPEZ_EINVAL;
    const uint64_t nb = n_blocks(d, c);
    for (uint64_t b = 0; b < nb; b++)
      if (c->block_cfg[b] >= c->n_cand) return HPEZ_EINVAL;
  }
  return HPEZ_OK;
}

uint64_t n_blocks(const hpez_field_desc* d, const hpez_config* c)
{
  if (!c->block_log2) return 0;
  const uint64_t B = 1ull << c->block_log2;
  uint64_t nb = 1;
  for (int i = 0; i < d->ndims; i++) nb *= (d->dims[i] + B - 1) / B;
  return nb;
}

Geom make_geom(const hpez_field_desc* d, int frozen)
{
  Geom g;
  for (int i = 0; i < 4; i++) g.n[i] = i < d->ndims ? (int64_t)d->dims[i] : 1;
  g.st[3] = 1;
  for (int i = 2; i >= 0; i--) g.st[i] = g.st[i + 1] * g.n[i + 1];
  for (int i = 0; i < 4; i++) g.act[i] = (g.n[i] > 1 && i != frozen) ? 1 : 0;
  return g;
}

int n_active(const Geom& g)
{
  int k = 0;
  for (int i = 0; i < 4; i++) k += g.act[i];
  return k;
}

Lattice make_lattice(const Geom& g, const int64_t* r, const int64_t* m)
{
  Lattice L;
  L.total = 1;
  for (int d = 0; d < 4; d++) {
    L.first[d] = r[d];
    L.step[d] = m[d];
    L.cnt[d] = r[d] <= g.n[d] - 1 ? (uint32_t)((g.n[d] - 1 - r[d]) / m[d] + 1) : 0;
    L.total *= L.cnt[d];
  }
  return L;
}

// Eq. (15), level 1 always e.
double level_eb(double e, double alpha, double beta, int l)
{
  double pw = 1.0;
  for (int i = 1; i < l; i++) pw = pw * alpha;
  double m = pw < beta ? pw : beta;
  if (l == 1) m = 1.0;
  return e / m;
}

uint64_t anchors_of(const Geom& g, int anchor_log2)
{
  const int64_t A = (int64_t)1 << anchor_log2;
  uint64_t c = 1;
  for (int d = 0; d < 4; d++) c *= g.act[d] ? (uint64_t)((g.n[d] - 1) / A + 1) : (uint64_t)g.n[d];
  return c;
}

static uint64_t al8(uint64_t v) { return (v + 7) & ~7ull; }

void layout(Layout* L, uint64_t s)
{
  uint64_t t = kHdrBytes;
  L->off_blocks = t;
  t = al8(t + L->n_blocks);
  L->off_anchor = t;
  t = al8(t + L->n_anchor * s);
  L->off_unpred = t;
  t = al8(t + L->n_unpred * s);
  L->off_outl = t;
  t = al8(t + L->n_outlier * 8);
  L->off_pidx = t;
  t = al8(t + L->n_patch * 8);
  L->off_pval = t;
  t = al8(t + L->n_patch * s);
  L->off_len = t;
  t = al8(t + (L->sym_max >= L->sym_min ? (uint64_t)(L->sym_max - L->sym_min + 1) : 0));
  L->off_chunks = t;
  t = al8(t + L->n_chunks * 2);
  L->off_payload = t;
  t += ((L->payload_bits + 31) / 32) * 4;
  L->total = t;
}

static void put_interp(uint8_t* h, const hpez_interp& c)
{
  h[0] = c.kind;
  h[1] = c.md;
  h[2] = c.same_level;
  for (int j = 0; j < 4; j++) h[3 + j] = c.order[j];
  h[7] = 0;
}

void write_header(uint8_t* h, const hpez_field_desc* d, const hpez_config* c, const Layout& L)
{
  std::memset(h, 0, kHdrBytes);
  const uint32_t magic = kMagic;
  const uint16_t ver = 1;
  std::memcpy(h, &magic, 4);
  std::memcpy(h + 4, &ver, 2);
  h[6] = d->dtype;
  h[7] = d->ndims;
  for (int i = 0; i < 4; i++) {
    const uint64_t v = i < d->ndims ? d->dims[i] : 1;
    std::memcpy(h + 8 + 8 * i, &v, 8);
  }
  h[40] = d->eb_mode;
  h[41] = L.predictor;
  h[42] = c->anchor_log2;
  h[43] = (uint8_t)c->frozen_dim;
  h[44] = c->block_log2;
  h[45] = (uint8_t)c->n_cand;
  h[46] = (uint8_t)kBrickLog2;
  std::memcpy(h + 48, &c->radius, 4);
  std::memcpy(h + 52, &c->chunk, 4);
  std::memcpy(h + 56, &d->eb, 8);
  std::memcpy(h + 64, &L.e, 8);
  std::memcpy(h + 72, &c->alpha, 8);
  std::memcpy(h + 80, &c->beta, 8);
  std::memcpy(h + 88, c->md_w, 96);
  for (int i = 0; i < 16; i++) put_interp(h + 184 + 8 * i, c->level[i]);
  for (int i = 0; i < 16; i++) {
    hpez_interp z;
    std::memset(&z, 0, sizeof z);
    for (int j = 0; j < 4; j++) z.order[j] = (uint8_t)j;
    put_interp(h + 312 + 8 * i, (uint32_t)i < c->n_cand ? c->cand[i] : z);
  }
  std::memcpy(h + 440, &L.n_blocks, 8);
  std::memcpy(h + 448, &L.n_anchor, 8);
  std::memcpy(h + 456, &L.n_unpred, 8);
  std::memcpy(h + 464, &L.n_outlier, 8);
  std::memcpy(h + 472, &L.n_patch, 8);
  std::memcpy(h + 480, &L.sym_min, 4);
  std::memcpy(h + 484, &L.sym_max, 4);
  std::memcpy(h + 488, &L.n_chunks, 8);
  std::memcpy(h + 496, &L.payload_bits, 8);
  std::memcpy(h + 504, &L.total, 8);
}

int read_header(const uint8_t* h, uint64_t n, hpez_field_desc* d, hpez_config* c, Layout* L)
{
  if (n < (uint64_t)kHdrBytes) return HPEZ_ECORRUPT;
  uint32_t magic;
  uint16_t ver;
  std::memcpy(&magic, h, 4);
  std::memcpy(&ver, h + 4, 2);
  if (magic != kMagic || ver != 1) return HPEZ_ECORRUPT;
  std::memset(d, 0, sizeof *d);
  std::memset(c, 0, sizeof *c);
  std::memset(L, 0, sizeof *L);
  d->dtype = h[6];
  d->ndims = h[7];
  for (int i = 0; i < 4; i++) std::memcpy(&d->dims[i], h + 8 + 8 * i, 8);
  d->eb_mode = h[40];
  L->predictor = h[41];
  c->predictor = L->predictor == 1 ? 1 : 0;
  c->anchor_log2 = h[42];
  c->frozen_dim = (int8_t)h[43];
  c->block_log2 = h[44];
  c->n_cand = h[45];
  if (h[46] != kBrickLog2 || h[47] != 0) return HPEZ_ECORRUPT;
  std::memcpy(&c->radius, h + 48, 4);
  std::memcpy(&c->chunk, h + 52, 4);
  std::memcpy(&d->eb, h + 56, 8);
  std::memcpy(&L->e, h + 64, 8);
  std::memcpy(&c->alpha, h + 72, 8);
  std::memcpy(&c->beta, h + 80, 8);
  std::memcpy(c->md_w, h + 88, 96);
  for (int i = 0; i < 16; i++) {
    const uint8_t* p = h + 184 + 8 * i;
    c->level[i].kind = p[0];
    c->level[i].md = p[1];
    c->level[i].same_level = p[2];
    for (int j = 0; j < 4; j++) c->level[i].order[j] = p[3 + j];
  }
  for (int i = 0; i < 16; i++) {
    const uint8_t* p = h + 312 + 8 * i;
    c->cand[i].kind = p[0];
    c->cand[i].md = p[1];
    c->cand[i].same_level = p[2];
    for (int j = 0; j < 4; j++) c->cand[i].order[j] = p[3 + j];
  }
  std::memcpy(&L->n_blocks, h + 440, 8);
  std::memcpy(&L->n_anchor, h + 448, 8);
  std::memcpy(&L->n_unpred, h + 456, 8);
  std::memcpy(&L->n_outlier, h + 464, 8);
  std::memcpy(&L->n_patch, h + 472, 8);
  std::memcpy(&L->sym_min, h + 480, 4);
  std::memcpy(&L->sym_max, h + 484, 4);
  std::memcpy(&L->n_chunks, h + 488, 8);
  std::memcpy(&L->payload_bits, h + 496, 8);
  uint64_t total;
  std::memcpy(&total, h + 504, 8);
  if (L->predictor > 2) return HPEZ_ECORRUPT;
  if (check_desc(d) != HPEZ_OK) return HPEZ_ECORRUPT;
  if (check_cfg(d, c, false) != HPEZ_OK) return HPEZ_ECORRUPT;
  if (c->block_log2 && c->n_cand < 1) return HPEZ_ECORRUPT;
  const uint64_t N = points_of(d);
  if (L->n_blocks != n_blocks(d, c)) return HPEZ_ECORRUPT;
  if (L->n_anchor > N || L->n_unpred > N || L->n_outlier > N || L->n_patch > N)
    return HPEZ_ECORRUPT;
  if (L->predictor != 2) {
    if (L->sym_max >= 2 * c->radius) return HPEZ_ECORRUPT;
    if (L->sym_min > L->sym_max && N > 0) return HPEZ_ECORRUPT;
    if (L->n_chunks != (N + c->chunk - 1) / c->chunk) return HPEZ_ECORRUPT;
    if (L->payload_bits > N * (uint64_t)kLmax) return HPEZ_ECORRUPT;
  }
  layout(L, d->dtype ? 8 : 4);
  if (L->total != total) return HPEZ_ECORRUPT;
  return HPEZ_OK;
}

// ---------------------------------------------------------------------------
// Huffman codebook on the host (Sec. 4, step 4): two-queue construction with
// leaf-first ties, count halving until the longest code fits 32 bits,
// canonical codewords by (length, symbol).

int huffman_lengths(const uint32_t* hist, uint32_t nsym, uint8_t* len)
{
  std::memset(len, 0, nsym);
  struct Leaf {
    uint64_t w;
    uint32_t sym;
  };
  std::vector<uint64_t> cnt(nsym);
  for (uint32_t i = 0; i < nsym; i++) cnt[i] = hist[i];
  std::vector<Leaf> leaves;
  for (uint32_t i = 0; i < nsym; i++)
    if (cnt[i]) leaves.push_back({cnt[i], i});
  const size_t K = leaves.size();
  if (K == 0) return HPEZ_OK;
  if (K == 1) {
    len[leaves[0].sym] = 1;
    return HPEZ_OK;
  }
  std::vector<uint64_t> w(2 * K);
  std::vector<uint32_t> left(K), right(K), depth(2 * K);
  for (;;) {
    leaves.clear();
    for (uint32_t i = 0; i < nsym; i++)
      if (cnt[i]) leaves.push_back({cnt[i], i});
    std::sort(leaves.begin(), leaves.end(), [](const Leaf& a, const Leaf& b) {
      return a.w != b.w ? a.w < b.w : a.sym < b.sym;
    });
    for (size_t i = 0; i < K; i++) w[i] = leaves[i].w;
    size_t q1 = 0, q2 = K, made = 0;
    auto pop = [&]() -> uint32_t {
      bool leaf;
      if (q1 >= K) leaf = false;
      else if (q2 >= K + made) leaf = true;
      else leaf = w[q1] <= w[q2];
      return (uint32_t)(leaf ? q1++ : q2++);
    };
    for (size_t m = 0; m + 1 < K; m++) {
      const uint32_t a = pop();
      const uint32_t b = pop();
      w[K + made] = w[a] + w[b];
      left[made] = a;
      right[made] = b;
      made++;
    }
    const size_t root = K + made - 1;
    depth[root] = 0;
    uint32_t maxd = 0;
    for (size_t node = root + 1; node-- > K;) {
      const uint32_t kids[2] = {left[node - K], right[node - K]};
      for (uint32_t ch : kids) {
        depth[ch] = depth[node] + 1;
        if (ch < K) maxd = std::max(maxd, depth[ch]);
      }
    }
    if (maxd <= (uint32_t)kLmax) {
      for (size_t i = 0; i < K; i++) len[leaves[i].sym] = (uint8_t)depth[i];
      return HPEZ_OK;
    }
    for (uint32_t i = 0; i < nsym; i++)
      if (cnt[i]) cnt[i] = (cnt[i] + 1) >> 1;
  }
}

void canonical_codes(const uint8_t* len, uint32_t nsym, uint32_t* cw)
{
  // count per length, then first codeword per length, then assign in symbol order
  uint32_t nl[kLmax + 1] = {0};
  for (uint32_t s = 0; s < nsym; s++)
    if (len[s]) nl[len[s]]++;
  uint64_t next[kLmax + 2] = {0};
  uint64_t code = 0;
  int prev = 0;
  bool any = false;
  for (int l = 1; l <= kLmax; l++) {
    if (!nl[l]) continue;
    code = any ? (code + 1) << (l - prev) : 0;
    next[l] = code;
    code += nl[l] - 1;
    prev = l;
    any = true;
  }
  for (uint32_t s = 0; s < nsym; s++) cw[s] = len[s] ? (uint32_t)next[len[s]]++ : 0;
}

int encode_payload(hpez_ctx* ctx, const uint16_t* code, uint64_t N, uint32_t chunk,
                   const uint8_t* h_len, const uint32_t* h_cw, uint32_t sym_min, uint32_t sym_max,
                   const uint8_t* dlen, const uint32_t* dcw, uint32_t* d_tab, uint64_t* d_flags,
                   uint32_t* d_ticket, uint32_t* h_tab, uint32_t* payload, uint16_t* chunks,
                   hipStream_t st)
{
  const uint64_t nch = (N + chunk - 1) / chunk;
  if (!nch) return HPEZ_OK;
  if (sym_max < sym_min) return HPEZ_EINVAL;
  EncodeArgs a;
  std::memset(&a, 0, sizeof a);
  a.n = N;
  a.nch = nch;
  a.chunk = chunk;
  a.smin = sym_min;
  a.ntab = sym_max - sym_min + 1;
  a.lds_tab = a.ntab <= kEncTab;
  // packed entries (codeword << 6 | length) need codewords of at most 26 bits
  uint32_t maxlen = 0;
  for (uint32_t k = sym_min; k <= sym_max; k++) maxlen = std::max<uint32_t>(maxlen, h_len[k]);
  a.packed_ok = maxlen <= 26;
  if (a.packed_ok) {
    for (uint32_t k = 0; k < a.ntab; k++)
      h_tab[k] = h_len[sym_min + k] ? (h_cw[sym_min + k] << 6 | h_len[sym_min + k]) : 0u;
    if (hipMemcpyAsync(d_tab, h_tab, (size_t)a.ntab * 4, hipMemcpyHostToDevice, st) != hipSuccess)
      return HPEZ_EDEVICE;
  }
  if (hipMemsetAsync(d_flags, 0, nch * 8, st) != hipSuccess) return HPEZ_EDEVICE;
  if (hipMemsetAsync(d_ticket, 0, 4, st) != hipSuccess) return HPEZ_EDEVICE;
  hipEvent_t ev = ctx_span_begin(ctx, st);
  if (launch_encode1(a, code, payload, chunks, d_flags, d_ticket, d_tab, dlen, dcw, st) !=
      hipSuccess)
    return HPEZ_EDEVICE;
  ctx_span_end(ctx, ev, "encode", N * 2, st);
  return HPEZ_OK;
}

// Decode tables: 12-bit lookup (sym << 8 | len) plus per-length first code,
// count and offset into the (length, symbol)-sorted symbol list.
void decode_tables(const uint8_t* len, uint32_t nsym, uint32_t* lut, uint16_t* sorted,
                   uint64_t* lim, uint32_t* base)
{
  uint64_t count[kLmax + 2] = {0}, next[kLmax + 2] = {0}, offset[kLmax + 2] = {0};
  for (uint32_t s = 0; s < nsym; s++)
    if (len[s]) count[len[s]]++;
  // canonical first code per length, lengths without codes included
  for (int l = 2; l <= kLmax; l++) next[l] = (next[l - 1] + count[l - 1]) << 1;
  for (int l = 2; l <= kLmax; l++) offset[l] = offset[l - 1] + count[l - 1];
  lim[0] = 0;
  base[0] = 0;
  for (int l = 1; l <= kLmax; l++) {
    lim[l] = (next[l] + count[l]) << (32 - l);
    base[l] = (uint32_t)(offset[l] - next[l]);
  }
  std::memset(lut, 0, sizeof(uint32_t) << kLutBits);
  uint64_t fill[kLmax + 2];
  for (int l = 0; l <= kLmax + 1; l++) fill[l] = 0;
  for (uint32_t s = 0; s < nsym; s++) {
    const int l = len[s];
    if (!l) continue;
    const uint64_t rank = fill[l]++;
    sorted[offset[l] + rank] = (uint16_t)s;
    if (l <= kLutBits) {
      const uint64_t first = (next[l] + rank) << (kLutBits - l);
      for (uint64_t j = 0; j < (1ull << (kLutBits - l)); j++) lut[first + j] = (s << 8) | (uint32_t)l;
    }
  }
}

// MD weight table: [kind][odd set][dim] = md_w[kind][d] / sum over the odd set
// (ascending dims), Eq. (12).
void md_table(const hpez_config* c, double* wq)
{
  for (int k = 0; k < 3; k++)
    for (unsigned odd = 0; odd < 16; odd++) {
      double sum = 0.0;
      for (int d = 0; d < 4; d++)
        if (odd >> d & 1u) sum = sum + c->md_w[k][d];
      for (int d = 0; d < 4; d++)
        wq[(k * 16 + odd) * 4 + d] = (odd >> d & 1u) ? c->md_w[k][d] / sum : 0.0;
    }
}

}  // namespace hpez

// ---------------------------------------------------------------------------
// context and workspace

#define HIPCK(x)                        \
  do {                                  \
    if ((x) != hipSuccess) return HPEZ_EDEVICE; \
  } while (0)

namespace {

struct Bump {
  uint8_t* base;
  size_t off = 0;
  template <typename U>
  U* take(size_t count)
  {
    off = (off + 255) & ~(size_t)255;
    U* p = reinterpret_cast<U*>(base + off);
    off += count * sizeof(U);
    return p;
  }
};

int ensure_ws(hpez_ctx* ctx, size_t bytes)
{
  if (bytes <= ctx->ws_bytes) return HPEZ_OK;
  if (ctx->ws) (void)hipFree(ctx->ws);
  ctx->ws = nullptr;
  ctx->ws_bytes = 0;
  const size_t want = bytes + (bytes >> 4);
  if (hipMalloc(&ctx->ws, want) != hipSuccess) {
    ctx->ws = nullptr;
    return HPEZ_ENOMEM;
  }
  ctx->ws_bytes = want;
  return HPEZ_OK;
}

int ensure_pinned(hpez_ctx* ctx, size_t bytes)
{
  if (bytes <= ctx->pinned_bytes) return HPEZ_OK;
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  ctx->pinned = nullptr;
  ctx->pinned_bytes = 0;
  if (hipHostMalloc((void**)&ctx->pinned, bytes, hipHostMallocDefault) != hipSuccess) {
    ctx->pinned = nullptr;
    return HPEZ_ENOMEM;
  }
  ctx->pinned_bytes = bytes;
  return HPEZ_OK;
}

int ensure_pin_tab(hpez_ctx* ctx, size_t bytes)
{
  if (bytes <= ctx->pin_tab_bytes) return HPEZ_OK;
  if (ctx->pin_tab) (void)hipHostFree(ctx->pin_tab);
  ctx->pin_tab = nullptr;
  ctx->pin_tab_bytes = 0;
  if (hipHostMalloc((void**)&ctx->pin_tab, bytes, hipHostMallocDefault) != hipSuccess) {
    ctx->pin_tab = nullptr;
    return HPEZ_ENOMEM;
  }
  ctx->pin_tab_bytes = bytes;
  return HPEZ_OK;
}

struct DevScope {
  int prev = -1;
  explicit DevScope(int dev)
  {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DevScope()
  {
    int cur = prev;
    if (hipGetDevice(&cur) != hipSuccess) return;
    if (prev >= 0 && cur != prev) (void)hipSetDevice(prev);
  }
};

// Workspace needed by compress/decompress of N points.
size_t ws_need(uint64_t N, uint64_t s, uint32_t R, uint32_t chunk, uint64_t nb, int op)
{
  const uint64_t nch = (N + chunk - 1) / chunk;
  const uint64_t nsym = 2ull * R;
  size_t b = 0;
  auto add = [&](size_t v) { b += (v + 255) & ~(size_t)255; b += 256; };
  if (op == 0) add(N * s);                 // W
  add(N * 2);                              // codes
  add(nsym * 4);                           // histogram
  add(nsym);                               // lengths
  add(nsym * 4);                           // codewords
  add(nch * 4 * 2);                        // chunk bits, chunk zeros
  add((nch + 1) * 8 * 2);                  // offsets (+ totals)
  add(((nch + 1023) / 1024 + 1) * 8 * 2);  // scan tiles
  add(2 * 1024 * 8 + 64);                  // min/max partials
  add(N * s);                              // anchors staging (bounded by N)
  add(nb + 16);                            // block configs
  add(3 * 16 * 4 * 8);                     // MD weights
  add((1u << kLutBits) * 4 + 4 * 34 * 4 + nsym * 2);  // decode tables
  add(64);                                 // status
  add(64);                                 // encoder ticket
  return b;
}

// points of the grid of stride s (multiples of s on active dims)
uint64_t grid_points(const Geom& g, int64_t s)
{
  uint64_t p = 1;
  for (int d = 0; d < 4; d++) p *= g.act[d] ? (uint64_t)((g.n[d] - 1) / s + 1) : (uint64_t)g.n[d];
  return p;
}

template <typename T>
int run_levels(hpez_ctx* ctx, const hpez_field_desc* d, const hpez_config* c, const Geom& g,
               double e, const T* X, T* W, uint16_t* code, const uint8_t* d_bcfg,
               const double* d_wq, const double* h_wq, int mode, hipStream_t st, int l_stop = 0)
{
  const int L = c->anchor_log2;
  const int64_t B = c->block_log2 ? (int64_t)1 << c->block_log2 : 0;
  const int nact = n_active(g);
  for (int l = L; l > l_stop; l--) {
    const int64_t s = (int64_t)1 << (l - 1);
    // algorithmic traffic of the level: each of its points reads its value
    // (original or code) once and writes its code or reconstruction once
    const uint64_t pts = grid_points(g, s) - grid_points(g, 2 * s);
    Span span(ctx, mode == 0 ? (l == 1 ? "predict_l1" : "predict_coarse")
                             : (l == 1 ? "reconstruct_l1" : "reconstruct_coarse"),
              pts * (sizeof(T) + 2), st);
    const double el = level_eb(e, c->alpha, c->beta, l);
    const double inv2e = 1.0 / (2.0 * el), twoe = 2.0 * el;
    const hpez_interp& ip = c->level[l - 1];
    const bool blocks = B > 0 && s < B;
    StepArgs a;
    std::memset(&a, 0, sizeof a);
    a.g = g;
    a.s = s;
    a.B = B;
    a.filter = blocks ? 1 : 0;
    a.kind = ip.kind;
    a.md = ip.md;
    a.el = el;
    a.inv2e = inv2e;
    a.twoe = twoe;
    a.R = c->radius;
    int64_t r[4], m[4];
    if (ip.md) {
      for (int cnt = 1; cnt <= nact; cnt++)
        for (unsigned odd = 1; odd < 16; odd++) {
          bool ok = (int)__builtin_popcount(odd) == cnt;
          for (int dd = 0; dd < 4; dd++)
            if ((odd >> dd & 1u) && !g.act[dd]) ok = false;
          if (!ok) continue;
          for (int dd = 0; dd < 4; dd++) {
            if (!g.act[dd]) { r[dd] = 0; m[dd] = 1; }
            else if (odd >> dd & 1u) { r[dd] = s; m[dd] = 2 * s; }
            else { r[dd] = 0; m[dd] = 2 * s; }
          }
          a.lat = make_lattice(g, r, m);
          a.odd = odd;
          for (int dd = 0; dd < 4; dd++) a.wq[dd] = h_wq[(ip.kind * 16 + odd) * 4 + dd];
          HIPCK(launch_step<T>(a, X, W, code, mode, st));
        }
    } else {
      int pos[4] = {-1, -1, -1, -1}, np = 0;
      for (int i = 0; i < 4; i++) {
        const int dd = ip.order[i];
        if (dd < 4 && g.act[dd] && pos[dd] < 0) pos[dd] = np++;
      }
      for (int k = 0; k < np; k++) {
        int pd = 0;
        for (int dd = 0; dd < 4; dd++)
          if (pos[dd] == k) pd = dd;
        for (int dd = 0; dd < 4; dd++) {
          if (!g.act[dd]) { r[dd] = 0; m[dd] = 1; }
          else if (dd == pd) { r[dd] = s; m[dd] = 2 * s; }
          else if (pos[dd] < k) { r[dd] = 0; m[dd] = s; }
          else { r[dd] = 0; m[dd] = 2 * s; }
        }
        a.pdim = pd;
        if (ip.kind != 0 && ip.same_level) {
          m[pd] = 4 * s;
          r[pd] = s;
          a.sl = 0;
          a.lat = make_lattice(g, r, m);
          HIPCK(launch_step<T>(a, X, W, code, mode, st));
          r[pd] = 3 * s;
          a.sl = 1;
          a.lat = make_lattice(g, r, m);
          HIPCK(launch_step<T>(a, X, W, code, mode, st));
          a.sl = 0;
        } else {
          a.sl = 0;
          a.lat = make_lattice(g, r, m);
          HIPCK(launch_step<T>(a, X, W, code, mode, st));
        }
      }
    }
    if (blocks) {
      BlockStepArgs bsa;
      std::memset(&bsa, 0, sizeof bsa);
      bsa.g = g;
      bsa.s = s;
      bsa.B = B;
      for (int dd = 0; dd < 4; dd++) bsa.nb[dd] = (g.n[dd] + B - 1) / B;
      for (int dd = 0; dd < 4; dd++) {
        r[dd] = 0;
        m[dd] = g.act[dd] ? s : 1;
      }
      bsa.lat = make_lattice(g, r, m);
      bsa.el = el;
      bsa.inv2e = inv2e;
      bsa.twoe = twoe;
      bsa.R = c->radius;
      for (uint32_t i = 0; i < c->n_cand; i++) bsa.cand[i] = c->cand[i];
      for (int t = 0; t < 2 * nact; t++) {
        bsa.t = t;
        HIPCK(launch_block_step<T>(bsa, X, W, code, d_bcfg, d_wq, mode, st));
      }
    }
  }
  (void)d;
  return HPEZ_OK;
}

Lattice anchor_lattice(const Geom& g, int anchor_log2)
{
  int64_t r[4], m[4];
  const int64_t A = (int64_t)1 << anchor_log2;
  for (int d = 0; d < 4; d++) {
    r[d] = 0;
    m[d] = g.act[d] ? A : 1;
  }
  return make_lattice(g, r, m);
}

// Block-wise fast path of one field: face phase and per-block interiors.
// Workspace: block_fast_bytes + block_tables_bound(1) from bw.
template <typename T>
int block_phase(hpez_ctx* ctx, const hpez_config* c, const Geom& g, double e, const T* X,
                const T* Wg, uint16_t* code, const uint8_t* dbcfg, const double* h_wq,
                uint32_t* hist, uint32_t lo, T* out, int mode, Bump& bw, hipStream_t st)
{
  BlockJobHost<T> J;
  J.c = c;
  J.g = g;
  J.e = e;
  J.X = X;
  J.Wg = Wg;
  J.code = code;
  J.d_bcfg = dbcfg;
  J.h_wq = h_wq;
  J.hist = hist;
  J.hist_lo = lo;
  J.area = bw.take<uint8_t>(block_fast_bytes<T>(g));
  J.out = out;
  int rc = block_job_prepare<T>(ctx, J);
  if (rc) return rc;
  const size_t tb = block_jobs_table_bytes<T>(&J, 1);
  if (tb > block_tables_bound<T>(1)) return HPEZ_EINVAL;
  rc = ensure_pin_tab(ctx, tb);
  if (rc) return rc;
  void* dt = bw.take<uint8_t>(tb);
  return run_block_jobs<T>(ctx, &J, 1, mode, dt, ctx->pin_tab, st);
}

template <typename T>
int compress_t(hpez_ctx* ctx, const hpez_field_desc* d, const T* X, const hpez_config* c,
               uint8_t* out, uint64_t cap, uint64_t* out_size, hipStream_t st)
{
  const uint64_t N = points_of(d);
  const uint64_t s = sizeof(T);
  const uint32_t nsym = 2 * c->radius;
  const uint64_t nb = n_blocks(d, c);
  const Geom g = make_geom(d, c->frozen_dim);
  int rc = ensure_ws(ctx, ws_need(N, s, c->radius, c->chunk, nb, 0) + block_fast_bytes<T>(g) +
                             block_tables_bound<T>(1) + 512);
  if (rc) return rc;
  const size_t pin_need = (size_t)nsym * 4 + nsym + kHdrBytes + nb + 4096 + (size_t)nsym * 4;
  rc = ensure_pinned(ctx, pin_need);
  if (rc) return rc;
  Bump bw{(uint8_t*)ctx->ws};
  T* W = bw.take<T>(N);
  uint16_t* code = bw.take<uint16_t>(N);
  uint32_t* hist = bw.take<uint32_t>(nsym);
  uint8_t* dlen = bw.take<uint8_t>(nsym);
  uint32_t* dcw = bw.take<uint32_t>(nsym);
  const uint64_t nch = (N + c->chunk - 1) / c->chunk;
  uint32_t* cbits = bw.take<uint32_t>(nch + 1);
  uint32_t* czero = bw.take<uint32_t>(nch + 1);
  uint64_t* boff = bw.take<uint64_t>(nch + 1);
  uint64_t* zoff = bw.take<uint64_t>(nch + 1);
  uint64_t* tmp1 = bw.take<uint64_t>((nch + 1023) / 1024 + 1);
  uint64_t* tmp2 = bw.take<uint64_t>((nch + 1023) / 1024 + 1);
  double* part = bw.take<double>(2 * 1024);
  double* mm = bw.take<double>(4);
  int* bad = bw.take<int>(4);
  T* anc = bw.take<T>(N);
  uint8_t* dbcfg = bw.take<uint8_t>(nb + 16);
  double* dwq = bw.take<double>(3 * 16 * 4);
  uint32_t* ticket = bw.take<uint32_t>(16);

  uint8_t* pin = ctx->pinned;
  uint32_t* h_hist = (uint32_t*)pin;
  uint8_t* h_len = pin + (size_t)nsym * 4;
  uint8_t* h_hdr = h_len + nsym;
  double* h_mm = (double*)(h_hdr + kHdrBytes);
  int* h_bad = (int*)(h_mm + 2);
  uint32_t* h_tab = (uint32_t*)(pin + (((size_t)nsym * 5 + kHdrBytes + 64 + 63) & ~(size_t)63));

  // --- error bound (Sec. 7.1.3) and the non-finite check
  const int mblocks = 1024;
  HIPCK(hipMemsetAsync(bad, 0, sizeof(int), st));
  {
    Span sp(ctx, "minmax", N * s, st);
    HIPCK(launch_minmax<T>(X, N, part, bad, mblocks, st));
    HIPCK(launch_minmax_final(part, mblocks, mm, st));
  }
  HIPCK(hipMemcpyAsync(h_mm, mm, 16, hipMemcpyDeviceToHost, st));
  HIPCK(hipMemcpyAsync(h_bad, bad, 4, hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  if (*h_bad) return HPEZ_EINVAL;
  double e;
  Layout Lo;
  std::memset(&Lo, 0, sizeof Lo);
  Lo.n_blocks = nb;
  Lo.sym_min = 1;
  Lo.sym_max = 0;
  if (d->eb_mode == HPEZ_REL) {
    const double range = h_mm[1] - h_mm[0];
    if (range == 0) {
      // constant field: one value
      Lo.predictor = 2;
      Lo.n_anchor = 1;
      Lo.e = 0;
      layout(&Lo, s);
      if (Lo.total > cap) return HPEZ_ENOSPC;
      write_header(h_hdr, d, c, Lo);
      HIPCK(hipMemsetAsync(out, 0, Lo.total, st));
      HIPCK(hipMemcpyAsync(out, h_hdr, kHdrBytes, hipMemcpyHostToDevice, st));
      if (nb) HIPCK(hipMemcpyAsync(out + Lo.off_blocks, c->block_cfg, nb, hipMemcpyHostToDevice, st));
      HIPCK(hipMemcpyAsync(out + Lo.off_anchor, X, s, hipMemcpyDeviceToDevice, st));
      HIPCK(hipStreamSynchronize(st));
      *out_size = Lo.total;
      return HPEZ_OK;
    }
    e = d->eb * range;
  } else {
    e = d->eb;
  }
  if (!(e > 0)) return HPEZ_EINVAL;
  Lo.e = e;
  Lo.predictor = c->predictor;
  if (c->predictor == HPEZ_LORENZO)
    return lorenzo_compress<T>(ctx, d, X, c, e, out, cap, out_size, st);

  // --- interpolation predictor + quantization (Sec. 5, Sec. 4 step 3)
  double h_wq[3 * 16 * 4];
  md_table(c, h_wq);
  HIPCK(hipMemcpyAsync(dwq, h_wq, sizeof h_wq, hipMemcpyHostToDevice, st));
  if (nb) HIPCK(hipMemcpyAsync(dbcfg, c->block_cfg, nb, hipMemcpyHostToDevice, st));
  const Lattice al = anchor_lattice(g, c->anchor_log2);
  Lo.n_anchor = al.total;
  HIPCK(launch_anchors<T>(g, al, X, W, code, anc, c->radius, 0, st));
  const bool fast = block_fast_ok<T>(c, g);
  rc = run_levels<T>(ctx, d, c, g, e, X, W, code, dbcfg, dwq, h_wq, 0, st,
                     fast ? c->block_log2 : 0);
  if (rc) return rc;
  HIPCK(hipMemsetAsync(hist, 0, (size_t)nsym * 4, st));
  if (fast) {
    // faces, then block interiors with the brick histogram fused in
    uint32_t lo = c->radius > kBlockHistWin / 2 ? c->radius - kBlockHistWin / 2 : 0;
    if (lo + kBlockHistWin > nsym) lo = nsym > (uint32_t)kBlockHistWin ? nsym - kBlockHistWin : 0;
    rc = block_phase<T>(ctx, c, g, e, X, W, code, dbcfg, h_wq, hist, lo, nullptr, 0, bw, st);
    if (rc) return rc;
  }

  // --- histogram and codebook (Sec. 4 step 4)
  if (!fast) {
    Span sp(ctx, "histogram", N * 2, st);
    HIPCK(launch_histogram(code, N, hist, nsym, c->radius, st));
  }
  HIPCK(hipMemcpyAsync(h_hist, hist, (size_t)nsym * 4, hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  rc = huffman_lengths(h_hist, nsym, h_len);
  if (rc) return rc;
  std::vector<uint32_t> cw(nsym);
  canonical_codes(h_len, nsym, cw.data());
  uint64_t bits = 0;
  for (uint32_t k = 0; k < nsym; k++) bits += (uint64_t)h_hist[k] * h_len[k];
  for (uint32_t k = 0; k < nsym; k++)
    if (h_len[k]) { Lo.sym_min = k; break; }
  for (uint32_t k = nsym; k-- > 0;)
    if (h_len[k]) { Lo.sym_max = k; break; }
  Lo.n_unpred = h_hist[0];
  Lo.n_chunks = nch;
  Lo.payload_bits = bits;
  layout(&Lo, s);
  if (Lo.total > cap) return HPEZ_ENOSPC;
  write_header(h_hdr, d, c, Lo);
  HIPCK(hipMemcpyAsync(dlen, h_len, nsym, hipMemcpyHostToDevice, st));
  HIPCK(hipMemcpyAsync(dcw, cw.data(), (size_t)nsym * 4, hipMemcpyHostToDevice, st));

  // --- assemble the stream
  HIPCK(hipMemsetAsync(out, 0, Lo.total, st));
  HIPCK(hipMemcpyAsync(out, h_hdr, kHdrBytes, hipMemcpyHostToDevice, st));
  if (nb) HIPCK(hipMemcpyAsync(out + Lo.off_blocks, c->block_cfg, nb, hipMemcpyHostToDevice, st));
  HIPCK(hipMemcpyAsync(out + Lo.off_anchor, anc, Lo.n_anchor * s, hipMemcpyDeviceToDevice, st));
  if (Lo.sym_max >= Lo.sym_min)
    HIPCK(hipMemcpyAsync(out + Lo.off_len, h_len + Lo.sym_min, Lo.sym_max - Lo.sym_min + 1,
                         hipMemcpyHostToDevice, st));
  if (Lo.n_unpred) {
    // verbatim values in stream order (Sec. 4: unpredictable points)
    Span sp(ctx, "gather_unpred", N * 2 + Lo.n_unpred * s * 2, st);
    HIPCK(launch_gather_unpred<T>(code, N, c->chunk, czero, zoff, tmp2, X,
                                  (T*)(out + Lo.off_unpred), g, st));
  }
  rc = encode_payload(ctx, code, N, c->chunk, h_len, cw.data(), Lo.sym_min, Lo.sym_max, dlen, dcw,
                      hist, boff, ticket, h_tab, (uint32_t*)(out + Lo.off_payload),
                      (uint16_t*)(out + Lo.off_chunks), st);
  if (rc) return rc;
  HIPCK(hipStreamSynchronize(st));
  prof_collect(ctx);
  *out_size = Lo.total;
  return HPEZ_OK;
}

template <typename T>
int decompress_t(hpez_ctx* ctx, const hpez_field_desc* d, const hpez_config* c, const Layout& Lo,
                 const uint8_t* in, T* out, hipStream_t st)
{
  const uint64_t N = points_of(d);
  const uint64_t s = sizeof(T);
  const uint32_t nsym = 2 * c->radius;
  const uint64_t nb = Lo.n_blocks;
  const Geom g = make_geom(d, c->frozen_dim);
  int rc = ensure_ws(ctx, ws_need(N, s, c->radius, c->chunk, nb, 1) +
                              (Lo.predictor == 1 ? N * 8 + 256 : 0) + block_fast_bytes<T>(g) +
                              block_tables_bound<T>(1) + 512);
  if (rc) return rc;
  rc = ensure_pinned(ctx, (size_t)nsym + 4096 + nb + 64);
  if (rc) return rc;
  Bump bw{(uint8_t*)ctx->ws};
  uint16_t* code = bw.take<uint16_t>(N);
  const uint64_t nch = Lo.n_chunks;
  uint32_t* cbits = bw.take<uint32_t>(nch + 1);
  uint32_t* czero = bw.take<uint32_t>(nch + 1);
  uint64_t* boff = bw.take<uint64_t>(nch + 1);
  uint64_t* zoff = bw.take<uint64_t>(nch + 1);
  uint64_t* tmp1 = bw.take<uint64_t>((nch + 1023) / 1024 + 1);
  uint64_t* tmp2 = bw.take<uint64_t>((nch + 1023) / 1024 + 1);
  double* dwq = bw.take<double>(3 * 16 * 4);
  uint32_t* dlut = bw.take<uint32_t>(1u << kLutBits);
  uint16_t* dsorted = bw.take<uint16_t>(nsym);
  int* status = bw.take<int>(4);
  uint8_t* pin = ctx->pinned;
  uint8_t* h_len = pin;
  uint8_t* h_bcfg = pin + nsym;
  int* h_status = (int*)(pin + nsym + ((nb + 63) & ~63ull));

  if (Lo.predictor == 2) {
    // constant field
    HIPCK(hipMemcpyAsync(out, in + Lo.off_anchor, s, hipMemcpyDeviceToDevice, st));
    // broadcast by doubling copies
    uint64_t have = 1;
    while (have < N) {
      const uint64_t m = have < N - have ? have : N - have;
      HIPCK(hipMemcpyAsync(out + have, out, m * s, hipMemcpyDeviceToDevice, st));
      have += m;
    }
    HIPCK(hipStreamSynchronize(st));
    return HPEZ_OK;
  }
  // code lengths and block configurations to the host
  std::memset(h_len, 0, nsym);
  if (Lo.sym_max >= Lo.sym_min)
    HIPCK(hipMemcpyAsync(h_len + Lo.sym_min, in + Lo.off_len, Lo.sym_max - Lo.sym_min + 1,
                         hipMemcpyDeviceToHost, st));
  if (nb) HIPCK(hipMemcpyAsync(h_bcfg, in + Lo.off_blocks, nb, hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  for (uint64_t b = 0; b < nb; b++)
    if (h_bcfg[b] >= c->n_cand) return HPEZ_ECORRUPT;
  uint64_t kraft = 0, used = 0;
  for (uint32_t k = 0; k < nsym; k++) {
    if (h_len[k] > kLmax) return HPEZ_ECORRUPT;
    if (h_len[k]) {
      kraft += 1ull << (kLmax - h_len[k]);
      used++;
    }
  }
  if (N > 0 && !(kraft == (1ull << kLmax) || (used == 1 && kraft == (1ull << (kLmax - 1)))))
    return HPEZ_ECORRUPT;
  std::vector<uint32_t> lut(1u << kLutBits);
  std::vector<uint16_t> sorted(nsym);
  DecodeArgs da;
  std::memset(&da, 0, sizeof da);
  da.n = N;
  da.nch = nch;
  da.nbits = Lo.payload_bits;
  da.chunk = c->chunk;
  decode_tables(h_len, nsym, lut.data(), sorted.data(), da.lim, da.base);
  {
    uint32_t nshort = 0, nused = 0;
    for (uint32_t k = 0; k < nsym; k++) {
      nused += h_len[k] != 0;
      nshort += h_len[k] != 0 && h_len[k] <= kLutBits;
    }
    da.long_first = nshort;
    da.n_long = nused - nshort;
  }
  HIPCK(hipMemcpyAsync(dlut, lut.data(), lut.size() * 4, hipMemcpyHostToDevice, st));
  HIPCK(hipMemcpyAsync(dsorted, sorted.data(), sorted.size() * 2, hipMemcpyHostToDevice, st));
  double h_wq[3 * 16 * 4];
  md_table(c, h_wq);
  HIPCK(hipMemcpyAsync(dwq, h_wq, sizeof h_wq, hipMemcpyHostToDevice, st));
  HIPCK(hipMemsetAsync(status, 0, sizeof(int), st));
  // chunk offsets, decode
  {
    Span sp(ctx, "decode_offsets", nch * 2, st);
    HIPCK(launch_u16_to_u32((const uint16_t*)(in + Lo.off_chunks), nch, cbits, st));
    HIPCK(launch_scan_u32_to_u64(cbits, nch, boff, boff + nch, tmp1, st));
  }
  {
    Span sp(ctx, "decode", N * 2 + (Lo.payload_bits + 7) / 8, st);
    HIPCK(launch_decode2(da, (const uint32_t*)(in + Lo.off_payload), boff, dlut, dsorted, code,
                         czero, status, st));
  }
  HIPCK(launch_scan_u32_to_u64(czero, nch, zoff, zoff + nch, tmp2, st));
  uint64_t h_tot[2];
  if (Lo.predictor == 1) {
    // Lorenzo alternative: residuals, running sums, patches
    long long* v = bw.take<long long>(N);
    const Geom gl = make_geom(d, -1);
    {
      Span sp(ctx, "lorenzo_rebuild", N * (2 + s), st);
      HIPCK(launch_lorenzo_rebuild<T>(code, gl, N, c->radius, c->chunk, czero, zoff,
                                      (const long long*)(in + Lo.off_outl), Lo.n_outlier,
                                      (const uint64_t*)(in + Lo.off_pidx),
                                      (const T*)(in + Lo.off_pval), Lo.n_patch, 2.0 * Lo.e, v, out,
                                      status, st));
    }
    HIPCK(hipMemcpyAsync(h_status, status, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCK(hipMemcpyAsync(&h_tot[0], zoff + nch, 8, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    prof_collect(ctx);
    if (*h_status || h_tot[0] != Lo.n_outlier) return HPEZ_ECORRUPT;
    return HPEZ_OK;
  }
  if (Lo.n_unpred)
    HIPCK(launch_scatter_unpred2<T>(code, N, c->chunk, czero, zoff, (const T*)(in + Lo.off_unpred),
                                    Lo.n_unpred, out, status, g, st));
  const Lattice al = anchor_lattice(g, c->anchor_log2);
  if (al.total != Lo.n_anchor) return HPEZ_ECORRUPT;
  HIPCK(launch_anchors<T>(g, al, nullptr, out, code, (T*)(in + Lo.off_anchor), c->radius, 1, st));
  const bool fast = block_fast_ok<T>(c, g);
  rc = run_levels<T>(ctx, d, c, g, Lo.e, nullptr, out, code, in + Lo.off_blocks, dwq, h_wq, 1, st,
                     fast ? c->block_log2 : 0);
  if (rc) return rc;
  if (fast) {
    rc = block_phase<T>(ctx, c, g, Lo.e, nullptr, out, code, in + Lo.off_blocks, h_wq, nullptr, 0,
                        out, 1, bw, st);
    if (rc) return rc;
  }
  HIPCK(hipMemcpyAsync(h_status, status, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCK(hipMemcpyAsync(&h_tot[0], zoff + nch, 8, hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  prof_collect(ctx);
  if (*h_status) return HPEZ_ECORRUPT;
  if (h_tot[0] != Lo.n_unpred) return HPEZ_ECORRUPT;
  return HPEZ_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

const char* hpez_strerror(int code) { return err_text(code); }

int hpez_ctx_create(hpez_ctx** out, int device)
{
  if (!out) return HPEZ_EINVAL;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return HPEZ_EDEVICE;
  hpez_ctx* c = new (std::nothrow) hpez_ctx;
  if (!c) return HPEZ_ENOMEM;
  c->device = device;
  *out = c;
  return HPEZ_OK;
}

void hpez_ctx_destroy(hpez_ctx* ctx)
{
  if (!ctx) return;
  DevScope ds(ctx->device);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->pin_tab) (void)hipHostFree(ctx->pin_tab);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  delete ctx;
}

int hpez_config_default(const hpez_field_desc* d, hpez_config* c)
{
  if (check_desc(d) || !c) return HPEZ_EINVAL;
  std::memset(c, 0, sizeof *c);
  int big = 0;
  for (int i = 0; i < d->ndims; i++) big += d->dims[i] > 1;
  c->predictor = HPEZ_INTERP;
  c->anchor_log2 = big >= 3 ? 6 : big == 2 ? 7 : 8;
  c->block_log2 = 0;
  c->frozen_dim = -1;
  c->radius = 32768;
  c->chunk = 1024;
  c->alpha = 1.0;
  c->beta = 1.0;
  for (int k = 0; k < 3; k++)
    for (int j = 0; j < 4; j++) c->md_w[k][j] = 1.0;
  for (int i = 0; i < 16; i++) {
    c->level[i].kind = HPEZ_LINEAR;
    for (int j = 0; j < 4; j++) c->level[i].order[j] = (uint8_t)j;
  }
  for (int i = 0; i < 16; i++)
    for (int j = 0; j < 4; j++) c->cand[i].order[j] = (uint8_t)j;
  return HPEZ_OK;
}

int hpez_compress_bound(const hpez_field_desc* d, const hpez_config* c, uint64_t* out_bytes)
{
  if (check_desc(d) || !c || !out_bytes) return HPEZ_EINVAL;
  if (c->chunk < 64 || c->radius < 1 || c->radius > 32768) return HPEZ_EINVAL;
  const uint64_t N = points_of(d);
  const uint64_t s = d->dtype ? 8 : 4;
  const uint64_t nch = (N + c->chunk - 1) / c->chunk;
  uint64_t b = kHdrBytes + 8 * 8 + n_blocks(d, c) + 2ull * c->radius + 2 * nch + 4 * N + 8;
  if (c->predictor == HPEZ_LORENZO) b += N * 8 + N * (8 + s);
  else b += N * s;
  *out_bytes = b;
  return HPEZ_OK;
}

int hpez_footprint(const hpez_field_desc* d, const hpez_config* c, int op, uint64_t* bytes)
{
  if (check_desc(d) || !c || !bytes || op < 0 || op > 2) return HPEZ_EINVAL;
  const uint64_t N = points_of(d);
  *bytes = ws_need(N, d->dtype ? 8 : 4, c->radius ? c->radius : 32768, c->chunk ? c->chunk : 1024,
                   n_blocks(d, c), op == 1 ? 1 : 0);
  return HPEZ_OK;
}

int hpez_compress(hpez_ctx* ctx, const hpez_field_desc* d, const void* d_in,
                  const hpez_config* c, void* d_out, uint64_t out_cap, uint64_t* out_size,
                  hipStream_t stream)
{
  if (!ctx || !d_in || !d_out || !out_size) return HPEZ_EINVAL;
  int rc = check_desc(d);
  if (rc) return rc;
  rc = check_cfg(d, c, true);
  if (rc) return rc;
  DevScope ds(ctx->device);
  if (d->dtype == HPEZ_F32)
    return compress_t<float>(ctx, d, (const float*)d_in, c, (uint8_t*)d_out, out_cap, out_size,
                             stream);
  return compress_t<double>(ctx, d, (const double*)d_in, c, (uint8_t*)d_out, out_cap, out_size,
                            stream);
}

int hpez_inspect(const void* h_hdr, uint64_t n, hpez_field_desc* desc, uint64_t* n_points,
                 uint64_t* total_bytes)
{
  if (!h_hdr || !desc) return HPEZ_EINVAL;
  hpez_config c;
  Layout L;
  int rc = read_header((const uint8_t*)h_hdr, n, desc, &c, &L);
  if (rc) return rc;
  if (n_points) *n_points = points_of(desc);
  if (total_bytes) *total_bytes = L.total;
  return HPEZ_OK;
}

int hpez_decompress(hpez_ctx* ctx, const void* d_in, uint64_t in_size, void* d_out,
                    uint64_t out_cap, hipStream_t stream)
{
  if (!ctx || !d_in || !d_out) return HPEZ_EINVAL;
  if (in_size < (uint64_t)kHdrBytes) return HPEZ_ECORRUPT;
  DevScope ds(ctx->device);
  uint8_t hdr[kHdrBytes];
  HIPCK(hipMemcpyAsync(hdr, d_in, kHdrBytes, hipMemcpyDeviceToHost, stream));
  HIPCK(hipStreamSynchronize(stream));
  hpez_field_desc d;
  hpez_config c;
  Layout L;
  int rc = read_header(hdr, in_size, &d, &c, &L);
  if (rc) return rc;
  if (L.total > in_size) return HPEZ_ECORRUPT;
  const uint64_t N = points_of(&d);
  if (out_cap < N * (d.dtype ? 8 : 4)) return HPEZ_ENOSPC;
  if (d.dtype == HPEZ_F32)
    return decompress_t<float>(ctx, &d, &c, L, (const uint8_t*)d_in, (float*)d_out, stream);
  return decompress_t<double>(ctx, &d, &c, L, (const uint8_t*)d_in, (double*)d_out, stream);
}

int hpez_profile_enable(hpez_ctx* ctx, int on)
{
  if (!ctx) return HPEZ_EINVAL;
  ctx->prof = on != 0;
  ctx->stats.clear();
  ctx->pend.clear();
  ctx->ev_used = 0;
  return HPEZ_OK;
}

int hpez_profile_read(hpez_ctx* ctx, hpez_kernel_stat* out, int cap, int* n)
{
  if (!ctx || !n || (cap > 0 && !out)) return HPEZ_EINVAL;
  *n = (int)ctx->stats.size();
  for (int i = 0; i < cap && i < *n; i++) out[i] = ctx->stats[i];
  return HPEZ_OK;
}

}  // extern "C"

// helpers for the other translation units of the runtime
namespace hpez {

void* ctx_ws(hpez_ctx* c, size_t bytes, int* rc)
{
  *rc = ensure_ws(c, bytes);
  return *rc ? nullptr : c->ws;
}

uint8_t* ctx_pin(hpez_ctx* c, size_t bytes, int* rc)
{
  *rc = ensure_pinned(c, bytes);
  return *rc ? nullptr : c->pinned;
}

int ctx_device(hpez_ctx* c) { return c->device; }

hipEvent_t ctx_span_begin(hpez_ctx* c, hipStream_t st)
{
  if (!c->prof) return nullptr;
  hipEvent_t a = c->take_event();
  if (a && hipEventRecord(a, st) != hipSuccess) a = nullptr;
  return a;
}

void ctx_span_end(hpez_ctx* c, hipEvent_t a, const char* name, uint64_t bytes, hipStream_t st)
{
  if (!a) return;
  hipEvent_t b = c->take_event();
  if (b && hipEventRecord(b, st) == hipSuccess) c->pend.push_back({a, b, name, bytes});
}

void ctx_prof_collect(hpez_ctx* c) { prof_collect(c); }

}  // namespace hpez
