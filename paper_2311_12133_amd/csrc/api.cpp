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
#include <atomic>
#include <map>
#include <set>
#include <string>
#include <new>
#include <thread>
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
  size_t ws_limit = 0;  // 0: no cap on the workspace
  // a fixed context (hpez_decompress_noalloc): workspace and host staging are
  // given at set-up and never grown; a call that needs more fails with
  // HPEZ_ENOMEM before any device work, and no second stream is created
  bool fixed = false;
  uint8_t* pin_pre = nullptr;  // first bytes of the streams being decompressed
  size_t pin_pre_bytes = 0;
  hipEvent_t ev_sync = nullptr;  // host waits for part of a stream's work
  void* aux = nullptr;           // integer fields' float64 copies (ctx_aux)
  size_t aux_bytes = 0;
  // launch shapes (hpez_autotune): cached choices, the ones being tried, and
  // the keys looked up since `seen` was cleared
  std::map<uint64_t, uint32_t> tiles, tile_try;
  std::set<uint64_t> tile_seen;
  // second stream for work that can overlap the caller's stream, with the
  // events that fork it from and join it back to that stream
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // streams for the independent per-field work of a batch (ctx_fork_pool),
  // with the events that fork them from and join them back to the caller's
  // stream; made on first use
  static constexpr int kPool = 4;
  hipStream_t pool[kPool] = {};
  hipEvent_t pool_join[kPool] = {};
  hipEvent_t pool_fork = nullptr;
  int pool_n = 0;
  // recording a decompression plan (hpez_decompress_plan): the call repeats
  // the device work of the eager call just made on this context, whose host
  // results (headers, code lengths, block configurations) are still in its
  // staging; nothing is synchronised, fetched or allocated, and each stream's
  // end-of-call check is recorded in `checks` instead of being made
  bool capture = false;
  struct Check {
    int idx;              // the stream's index in the call
    const int* status;    // device status word
    const uint64_t* tot;  // device count of verbatim values (or outliers)
    uint64_t want;        // the count the header gives
  };
  std::vector<Check> checks;
  // kernel timing (hpez_profile_enable)
  bool prof = false;
  std::string prof_only;  // record only the spans of this group (empty: all)
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
    if (c && c->prof && (c->prof_only.empty() || c->prof_only == name_)) {
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
  if (!d || d->dtype > HPEZ_I32 || d->ndims < 1 || d->ndims > 4 || d->eb_mode > 1) return HPEZ_EINVAL;
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
  if (c->predictor == HPEZ_LORENZO && dtype_int(d->dtype)) return HPEZ_EUNSUPPORTED;
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
  // only the used symbols take part (the halving below keeps a count >= 1)
  uint32_t lo = 0;
  while (lo < nsym && !hist[lo]) lo++;
  if (lo == nsym) return HPEZ_OK;
  uint32_t hi = nsym - 1;
  while (!hist[hi]) hi--;
  struct Leaf {
    uint64_t w;
    uint32_t sym;
  };
  std::vector<Leaf> used;
  // zero bins skipped four at a time
  uint32_t i = lo;
  for (; i + 4 <= hi + 1; i += 4) {
    uint64_t w[2];
    std::memcpy(w, hist + i, 16);
    if (!(w[0] | w[1])) continue;
    for (uint32_t j = 0; j < 4; j++)
      if (hist[i + j]) used.push_back({hist[i + j], i + j});
  }
  for (; i <= hi; i++)
    if (hist[i]) used.push_back({hist[i], i});
  const size_t K = used.size();
  if (K == 1) {
    len[used[0].sym] = 1;
    return HPEZ_OK;
  }
  std::vector<Leaf> leaves(K);
  std::vector<uint64_t> w(2 * K);
  std::vector<uint32_t> left(K), right(K), depth(2 * K);
  for (;;) {
    leaves = used;
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
    for (Leaf& l : used) l.w = (l.w + 1) >> 1;
  }
}

void canonical_codes(const uint8_t* len, uint32_t nsym, uint32_t* cw)
{
  canonical_codes_range(len, 0, nsym, cw);
}

// the same for symbols [lo, hi) (len is zero outside); cw is written there only
void canonical_codes_range(const uint8_t* len, uint32_t lo, uint32_t hi, uint32_t* cw)
{
  // count per length, then first codeword per length, then assign in symbol order
  uint32_t nl[kLmax + 1] = {0};
  for_used(len, lo, hi, [&](uint32_t s) { nl[len[s]]++; });
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
  std::memset(cw + lo, 0, (size_t)(hi - lo) * 4);
  for_used(len, lo, hi, [&](uint32_t s) { cw[s] = (uint32_t)next[len[s]]++; });
}

int encode_payload(hpez_ctx* ctx, const uint16_t* code, uint64_t N, uint32_t chunk,
                   const uint8_t* h_len, const uint32_t* h_cw, uint32_t sym_min, uint32_t sym_max,
                   const uint8_t* dlen, const uint32_t* dcw, uint32_t* d_tab, uint32_t tab_words,
                   uint64_t* d_flags, uint32_t* d_ticket, uint32_t* h_tab, uint32_t* payload,
                   uint16_t* chunks, hipStream_t st)
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
  // packed entries: codeword << 6 | length up to 26 bits, longer codewords
  // escaped into a long table placed after the packed one (both must fit the
  // tab_words of d_tab and h_tab, else the unpacked path takes the full tables)
  uint32_t nlong = 0;
  for_used(h_len, sym_min, sym_max + 1, [&](uint32_t k) { nlong += h_len[k] > 26; });
  const uint64_t loff = ((uint64_t)a.ntab + 1) & ~1ull;  // 8-byte aligned, in words
  a.packed_ok = loff + 2 * (uint64_t)nlong <= tab_words;
  if (a.packed_ok) {
    std::memset(h_tab, 0, (size_t)loff * 4);
    uint64_t* lt = reinterpret_cast<uint64_t*>(h_tab + loff);
    uint32_t il = 0;
    for_used(h_len, sym_min, sym_max + 1, [&](uint32_t k) {
      if (h_len[k] <= 26) {
        h_tab[k - sym_min] = h_cw[k] << 6 | h_len[k];
      } else {
        lt[il] = (uint64_t)h_cw[k] << 6 | h_len[k];
        h_tab[k - sym_min] = il++ << 6 | 63u;
      }
    });
    a.ltab = nlong ? reinterpret_cast<const uint64_t*>(d_tab + loff) : nullptr;
    if (hipMemcpyAsync(d_tab, h_tab, (size_t)(loff + 2 * (uint64_t)nlong) * 4,
                       hipMemcpyHostToDevice, st) != hipSuccess)
      return HPEZ_EDEVICE;
  }
  if (hipMemsetAsync(d_flags, 0, nch * 8, st) != hipSuccess) return HPEZ_EDEVICE;
  if (hipMemsetAsync(d_ticket, 0, 4, st) != hipSuccess) return HPEZ_EDEVICE;
  hipEvent_t ev = ctx_span_begin(ctx, st, "encode");
  if (launch_encode1(a, code, payload, chunks, d_flags, d_ticket, d_tab, dlen, dcw, st) !=
      hipSuccess)
    return HPEZ_EDEVICE;
  ctx_span_end(ctx, ev, "encode", N * 2, st);
  return HPEZ_OK;
}

// The encoder alone, its packed codebook (and long table d_ltab when a
// codeword exceeds 26 bits, else nullptr) already on the device and its flags
// and ticket already zero.
int encode_payload_packed(hpez_ctx* ctx, const uint16_t* code, uint64_t N, uint32_t chunk,
                          uint32_t sym_min, uint32_t sym_max, const uint32_t* d_tab,
                          const uint64_t* d_ltab, uint64_t* d_flags, uint32_t* d_ticket,
                          uint32_t* payload, uint16_t* chunks, hipStream_t st)
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
  a.packed_ok = true;
  a.ltab = d_ltab;
  hipEvent_t ev = ctx_span_begin(ctx, st, "encode");
  if (launch_encode1(a, code, payload, chunks, d_flags, d_ticket, d_tab, nullptr, nullptr, st) !=
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
  decode_tables_range(len, 0, nsym, lut, sorted, lim, base);
}

// the same for symbols [lo, hi) (len is zero outside)
void decode_tables_range(const uint8_t* len, uint32_t lo, uint32_t hi, uint32_t* lut,
                         uint16_t* sorted, uint64_t* lim, uint32_t* base)
{
  uint64_t count[kLmax + 2] = {0}, next[kLmax + 2] = {0}, offset[kLmax + 2] = {0};
  for_used(len, lo, hi, [&](uint32_t s) { count[len[s]]++; });
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
  for_used(len, lo, hi, [&](uint32_t s) {
    const int l = len[s];
    const uint64_t rank = fill[l]++;
    sorted[offset[l] + rank] = (uint16_t)s;
    if (l <= kLutBits) {
      const uint64_t first = (next[l] + rank) << (kLutBits - l);
      for (uint64_t j = 0; j < (1ull << (kLutBits - l)); j++) lut[first + j] = (s << 8) | (uint32_t)l;
    }
  });
}

uint32_t decode_subtables(const uint8_t* len, uint32_t lo, uint32_t hi, uint32_t* lut,
                          uint32_t* sub, uint32_t cap)
{
  // canonical codewords as in decode_tables_range: by length, then symbol
  uint64_t count[kLmax + 2] = {0}, next[kLmax + 2] = {0};
  for_used(len, lo, hi, [&](uint32_t s) { count[len[s]]++; });
  for (int l = 2; l <= kLmax; l++) next[l] = (next[l - 1] + count[l - 1]) << 1;
  uint8_t lmax[1u << kLutBits];
  std::memset(lmax, 0, sizeof lmax);
  uint64_t fill[kLmax + 2];
  for (int l = 0; l <= kLmax + 1; l++) fill[l] = next[l];
  for_used(len, lo, hi, [&](uint32_t s) {
    const int l = len[s];
    const uint64_t cw = fill[l]++;
    if (l <= kLutBits) return;
    const uint32_t pre = (uint32_t)(cw >> (l - kLutBits));
    const int lc = l < kLutBits + kDecSubBits ? l : kLutBits + kDecSubBits;
    if (lc > lmax[pre]) lmax[pre] = (uint8_t)lc;
  });
  uint32_t off[1u << kLutBits];
  uint64_t total = 0;
  for (uint32_t p = 0; p < (1u << kLutBits); p++) {
    off[p] = (uint32_t)total;
    if (lmax[p]) total += 1ull << (lmax[p] - kLutBits);
  }
  if (total == 0 || total > cap) return 0;
  std::memset(sub, 0, (size_t)total * 4);  // entries no codeword covers decode as invalid
  for (int l = 0; l <= kLmax + 1; l++) fill[l] = next[l];
  for_used(len, lo, hi, [&](uint32_t s) {
    const int l = len[s];
    const uint64_t cw = fill[l]++;
    if (l <= kLutBits) return;
    const uint32_t pre = (uint32_t)(cw >> (l - kLutBits));
    const int lm = lmax[pre];
    if (l > lm) return;  // beyond the table depth: by the limits
    const uint64_t rest = cw & ((1ull << (l - kLutBits)) - 1);
    const uint64_t first = off[pre] + (rest << (lm - l));
    for (uint64_t j = 0; j < (1ull << (lm - l)); j++) sub[first + j] = (s << 8) | (uint32_t)l;
  });
  for (uint32_t p = 0; p < (1u << kLutBits); p++)
    if (lmax[p]) lut[p] = (off[p] << 8) | 0x80u | (uint32_t)(lmax[p] - kLutBits);
  return (uint32_t)total;
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
  if (ctx->fixed) return HPEZ_ENOMEM;
  if (ctx->ws_limit && bytes > ctx->ws_limit) return HPEZ_ENOMEM;
  if (ctx->ws) (void)hipFree(ctx->ws);
  ctx->ws = nullptr;
  ctx->ws_bytes = 0;
  size_t want = bytes + (bytes >> 4);
  if (ctx->ws_limit && want > ctx->ws_limit) want = ctx->ws_limit;
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
  if (ctx->fixed) return HPEZ_ENOMEM;
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

int ensure_pin_pre(hpez_ctx* ctx, size_t bytes)
{
  if (bytes <= ctx->pin_pre_bytes) return HPEZ_OK;
  if (ctx->fixed) return HPEZ_ENOMEM;
  if (ctx->pin_pre) (void)hipHostFree(ctx->pin_pre);
  ctx->pin_pre = nullptr;
  ctx->pin_pre_bytes = 0;
  if (hipHostMalloc((void**)&ctx->pin_pre, bytes, hipHostMallocDefault) != hipSuccess) {
    ctx->pin_pre = nullptr;
    return HPEZ_ENOMEM;
  }
  ctx->pin_pre_bytes = bytes;
  return HPEZ_OK;
}

int ensure_pin_tab(hpez_ctx* ctx, size_t bytes)
{
  if (bytes <= ctx->pin_tab_bytes) return HPEZ_OK;
  if (ctx->fixed) return HPEZ_ENOMEM;
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

// points of the grid of stride s (multiples of s on active dims)
uint64_t grid_points(const Geom& g, int64_t s)
{
  uint64_t p = 1;
  for (int d = 0; d < 4; d++) p *= g.act[d] ? (uint64_t)((g.n[d] - 1) / s + 1) : (uint64_t)g.n[d];
  return p;
}

// Odd block steps (second halves of same-level passes) have points only in
// blocks whose candidate uses same-level cubic: false when no block's does
// (h_bcfg: host copy of the block choices, or null to decide from the candidates).
bool block_halves_used(const hpez_config* c, const Geom& g, int64_t B, const uint8_t* h_bcfg)
{
  bool cand_h[256] = {};
  bool any = false;
  for (uint32_t i = 0; i < c->n_cand; i++)
    any |= cand_h[i] = c->cand[i].kind != 0 && c->cand[i].same_level;
  if (!any || !h_bcfg) return any;
  uint64_t nb = 1;
  for (int d = 0; d < 4; d++) nb *= (uint64_t)((g.n[d] + B - 1) / B);
  for (uint64_t b = 0; b < nb; b++)
    if (cand_h[h_bcfg[b]]) return true;
  return false;
}

template <typename T>
int run_levels(hpez_ctx* ctx, const hpez_field_desc* d, const hpez_config* c, const Geom& g,
               double e, const T* X, T* W, uint16_t* code, const uint8_t* d_bcfg,
               const uint8_t* h_bcfg, const double* d_wq, const double* h_wq, int mode,
               hipStream_t st, int l_stop = 0)
{
  const int L = c->anchor_log2;
  const int64_t B = c->block_log2 ? (int64_t)1 << c->block_log2 : 0;
  const int nact = n_active(g);
  int halves = -1;  // block_halves_used, once a level with blocks is reached
  for (int l = L; l > l_stop; l--) {
    const int64_t s = (int64_t)1 << (l - 1);
    // algorithmic traffic of the level: each of its points reads its value
    // (original or code) once and writes its code or reconstruction once
    const uint64_t pts = grid_points(g, s) - grid_points(g, 2 * s);
    Span span(ctx, mode == 0 ? (l == 1 ? "predict_l1" : "predict_coarse")
                             : (l == 1 ? "reconstruct_l1" : "reconstruct_coarse"),
              pts * (sizeof(T) + 2), st);
    const double el = level_eb(e, c->alpha, c->beta, l);
    const double inv2e = 1.0 / (2.0 * el), twoe = twoe_of(el, d->dtype);
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
          if (ip.kind != 0 && ip.same_level) {
            // same-level cubic inside MD: checkerboard colour 0, then colour 1
            // with the same-level stencils
            for (int half = 0; half < 2; half++) {
              a.sl = half;
              a.mdhalf = 1 + half;
              HIPCK(launch_step<T>(a, X, W, code, mode, st));
            }
            a.sl = 0;
            a.mdhalf = 0;
          } else {
            HIPCK(launch_step<T>(a, X, W, code, mode, st));
          }
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
      // level points per block, about 4096 of them per work-group
      uint64_t ppb = 1;
      for (int dd = 0; dd < 4; dd++) {
        const int64_t ext = B < g.n[dd] ? B : g.n[dd];
        ppb *= (uint64_t)(g.act[dd] ? ext / s : ext);
      }
      const uint64_t P = ppb / 4096;
      bsa.pieces = (uint32_t)(P < 1 ? 1 : P > 256 ? 256 : P);
      if (halves < 0) halves = block_halves_used(c, g, B, h_bcfg) ? 1 : 0;
      for (int t = 0; t < 2 * nact; t++) {
        if ((t & 1) && !halves) continue;
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

// Block-wise fast path of several fields: face phase and per-block interiors
// of every job in fused launches.  Tables come from bw (block_tables_bound).
template <typename T>
int block_phase(hpez_ctx* ctx, std::vector<BlockJobHost<T>>& jobs, int mode, Bump& bw,
                hipStream_t st)
{
  if (jobs.empty()) return HPEZ_OK;
  for (auto& J : jobs) {
    const int rc = block_job_prepare<T>(ctx, J);
    if (rc) return rc;
  }
  const int n = (int)jobs.size();
  const size_t tb = block_jobs_table_bytes<T>(jobs.data(), n);
  if (tb > block_tables_bound<T>(n)) return HPEZ_EINVAL;
  int rc = ensure_pin_tab(ctx, tb);
  if (rc) return rc;
  void* dt = bw.take<uint8_t>(tb);
  return run_block_jobs<T>(ctx, jobs.data(), n, mode, dt, ctx->pin_tab, st);
}

static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// bytes of each stream read with its header when decompressing
constexpr uint64_t kPrefixBytes = 64 * 1024;

// Run fn(i) for i in [0, n) on up to 16 host threads (host-only work of
// independent fields: codebooks, decode tables).
template <typename F>
void host_parallel(int n, F fn)
{
  unsigned nt = std::thread::hardware_concurrency();
  if (nt > 16) nt = 16;
  if (n <= 1 || nt <= 1) {
    for (int i = 0; i < n; i++) fn(i);
    return;
  }
  if ((int)nt > n) nt = (unsigned)n;
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; t++)
    th.emplace_back([&]() {
      for (int i = next++; i < n; i = next++) fn(i);
    });
  for (auto& t : th) t.join();
}

// ---------------------------------------------------------------------------
// Compression of one field as a job in phases (Sec. 4): error bound; anchors
// and levels with quantization; histogram; codebook; stream assembly and
// encode.  The plain call runs one job, the batch call many with one stream
// synchronization per phase for all of them and the block phase of every
// block-wise field in fused launches.  Each field takes the same steps either
// way, so its stream is the same.
template <typename T>
struct CJob {
  const hpez_field_desc* d = nullptr;
  const T* X = nullptr;
  const hpez_config* c = nullptr;
  uint8_t* out = nullptr;
  uint64_t cap = 0;
  int rc = HPEZ_OK;
  int kind = 0;  // 0 interpolation, 1 constant field (written), 2 Lorenzo (run after the rest)
  uint64_t N = 0, nb = 0, nch = 0;
  uint32_t nsym = 0;
  Geom g;
  Layout Lo;
  bool fast = false;
  uint32_t lo = 0;
  double h_wq[3 * 16 * 4];
  uint32_t maxlen = 0;  // longest code length
  bool early = false;   // verbatim values gathered before the codebook
  bool xface = false;   // family 2's face array prefilled with the field's values
  uint64_t off_unpred = 0;
  // device workspace
  T* W = nullptr;
  uint16_t* code = nullptr;
  uint32_t* hist = nullptr;
  uint8_t* dlen = nullptr;
  uint32_t* dcw = nullptr;
  uint32_t* czero = nullptr;
  uint64_t* boff = nullptr;
  uint64_t* zoff = nullptr;
  uint64_t* tmp2 = nullptr;
  double* part = nullptr;
  double* mm = nullptr;
  int* bad = nullptr;
  T* anc = nullptr;
  uint8_t* dbcfg = nullptr;
  double* dwq = nullptr;
  uint32_t* ticket = nullptr;
  void* area = nullptr;
  uint8_t* d_stage = nullptr;  // device copy of h_stage
  // pinned host staging
  uint8_t* h_stage = nullptr;  // header, block configurations, code lengths, codebook
  uint8_t* h_up = nullptr;     // block configurations and MD weights (layout of dbcfg)
  uint32_t* h_hist = nullptr;
  uint8_t* h_len = nullptr;
  uint8_t* h_hdr = nullptr;
  double* h_mm = nullptr;
  int* h_bad = nullptr;
  uint32_t* h_tab = nullptr;
  uint32_t* h_cw = nullptr;
};

constexpr int kMinmaxBlocks = 1024;

template <typename T>
void c_init(CJob<T>& J)
{
  J.N = points_of(J.d);
  J.nsym = 2 * J.c->radius;
  J.nb = n_blocks(J.d, J.c);
  J.g = make_geom(J.d, J.c->frozen_dim);
  J.nch = (J.N + J.c->chunk - 1) / J.c->chunk;
  J.fast = J.c->predictor == HPEZ_INTERP && block_fast_ok<T>(J.c, J.g);
  std::memset(&J.Lo, 0, sizeof J.Lo);
}

// staging of the stream's small sections: header and block configurations,
// code lengths and the packed codebook, each part padded to 8 bytes
template <typename T>
size_t c_stage_bytes(const CJob<T>& J)
{
  return kHdrBytes + J.nb + 8 + J.nsym + 8 + (size_t)J.nsym * 4 + 64;
}

template <typename T>
size_t c_dev_bytes(const CJob<T>& J)
{
  const uint64_t s = sizeof(T);
  size_t b = al256(J.N * s) + al256(J.N * 2) + al256(J.nsym * 4) + al256(J.nsym) +
             al256(J.nsym * 4) + al256((J.nch + 1) * 4) + 3 * al256((J.nch + 1) * 8) +
             al256(2 * kMinmaxBlocks * 8) + al256(32) + al256(16) + al256(J.N * s) +
             al256(al256(J.nb + 16) + 3 * 16 * 4 * 8) + al256(64) + al256(c_stage_bytes(J));
  if (J.fast) b += al256(block_fast_bytes<T>(J.g));
  return b + 256;
}

template <typename T>
size_t c_pin_bytes(const CJob<T>& J)
{
  return al256(J.nsym * 4) + al256(J.nsym) + al256(kHdrBytes) + al256(64) + 2 * al256(J.nsym * 4) +
         al256(c_stage_bytes(J)) + al256(al256(J.nb + 16) + 3 * 16 * 4 * 8) + 256;
}

template <typename T>
void c_take(CJob<T>& J, Bump& bw, Bump& pb)
{
  J.W = bw.take<T>(J.N);
  J.code = bw.take<uint16_t>(J.N);
  J.hist = bw.take<uint32_t>(J.nsym);
  J.dlen = bw.take<uint8_t>(J.nsym);
  J.dcw = bw.take<uint32_t>(J.nsym);
  J.czero = bw.take<uint32_t>(J.nch + 1);
  J.boff = bw.take<uint64_t>(J.nch + 1);
  J.zoff = bw.take<uint64_t>(J.nch + 1);
  J.tmp2 = bw.take<uint64_t>(J.nch + 1);
  J.part = bw.take<double>(2 * kMinmaxBlocks);
  J.mm = bw.take<double>(4);
  J.bad = bw.take<int>(4);
  J.anc = bw.take<T>(J.N);
  // block configurations, then the MD weights: one upload (h_up)
  J.dbcfg = bw.take<uint8_t>(al256(J.nb + 16) + sizeof J.h_wq);
  J.dwq = reinterpret_cast<double*>(J.dbcfg + al256(J.nb + 16));
  J.ticket = bw.take<uint32_t>(16);
  if (J.fast) J.area = bw.take<uint8_t>(block_fast_bytes<T>(J.g));
  J.d_stage = bw.take<uint8_t>(c_stage_bytes(J));
  J.h_stage = pb.take<uint8_t>(c_stage_bytes(J));
  J.h_up = pb.take<uint8_t>(al256(J.nb + 16) + sizeof J.h_wq);
  J.h_hist = pb.take<uint32_t>(J.nsym);
  J.h_len = pb.take<uint8_t>(J.nsym);
  J.h_hdr = pb.take<uint8_t>(kHdrBytes);
  J.h_mm = pb.take<double>(2);
  J.h_bad = (int*)(J.h_mm + 2);
  J.h_tab = pb.take<uint32_t>(J.nsym);
  J.h_cw = pb.take<uint32_t>(J.nsym);
}

// error bound (Sec. 7.1.3) and the non-finite check
template <typename T>
int c_minmax(hpez_ctx* ctx, CJob<T>& J, hipStream_t st)
{
  HIPCK(hipMemsetAsync(J.bad, 0, sizeof(int), st));
  {
    Span sp(ctx, "minmax", J.N * sizeof(T), st);
    if (J.fast && J.g.n[2] >= 64 && (uint64_t)J.g.n[0] * (uint64_t)J.g.n[1] < (1ull << 32)) {
      // (rows along dim 2 long enough for a wave each) the block path's face
      // steps then read the values of the face points with x2 on the face
      // lattice from family 2's compact array instead of strided rows
      HIPCK(launch_minmax_faces<T>(J.X, J.g, block_face_arrays<T>(J.g, J.area), J.part, J.bad,
                                   kMinmaxBlocks, st));
      J.xface = true;
    } else {
      HIPCK(launch_minmax<T>(J.X, J.N, J.part, J.bad, kMinmaxBlocks, st));
    }
    HIPCK(launch_minmax_final(J.part, kMinmaxBlocks, J.mm, st));
  }
  HIPCK(hipMemcpyAsync(J.h_mm, J.mm, 16, hipMemcpyDeviceToHost, st));
  HIPCK(hipMemcpyAsync(J.h_bad, J.bad, 4, hipMemcpyDeviceToHost, st));
  return HPEZ_OK;
}

// after the minmax sync: e, then the predictor up to the block phase
template <typename T>
int c_predict(hpez_ctx* ctx, CJob<T>& J, hipStream_t st)
{
  const hpez_field_desc* d = J.d;
  const hpez_config* c = J.c;
  const uint64_t s = sizeof(T);
  if (*J.h_bad) {
    J.rc = HPEZ_EINVAL;
    return HPEZ_OK;
  }
  Layout& Lo = J.Lo;
  Lo.n_blocks = J.nb;
  Lo.sym_min = 1;
  Lo.sym_max = 0;
  double e;
  if (d->eb_mode == HPEZ_REL) {
    const double range = J.h_mm[1] - J.h_mm[0];
    if (range == 0) {
      // constant field: one value
      J.kind = 1;
      Lo.predictor = 2;
      Lo.n_anchor = 1;
      Lo.e = 0;
      layout(&Lo, s);
      if (Lo.total > J.cap) {
        J.rc = HPEZ_ENOSPC;
        return HPEZ_OK;
      }
      write_header(J.h_hdr, d, c, Lo);
      HIPCK(hipMemsetAsync(J.out, 0, Lo.total, st));
      HIPCK(hipMemcpyAsync(J.out, J.h_hdr, kHdrBytes, hipMemcpyHostToDevice, st));
      if (J.nb)
        HIPCK(hipMemcpyAsync(J.out + Lo.off_blocks, c->block_cfg, J.nb, hipMemcpyHostToDevice, st));
      HIPCK(hipMemcpyAsync(J.out + Lo.off_anchor, J.X, s, hipMemcpyDeviceToDevice, st));
      return HPEZ_OK;
    }
    e = d->eb * range;
  } else {
    e = d->eb;
  }
  if (!(e > 0)) {
    J.rc = HPEZ_EINVAL;
    return HPEZ_OK;
  }
  Lo.e = e;
  Lo.predictor = c->predictor;
  if (c->predictor == HPEZ_LORENZO) {
    J.kind = 2;
    return HPEZ_OK;
  }
  // interpolation predictor + quantization (Sec. 5, Sec. 4 step 3)
  md_table(c, J.h_wq);
  if (J.nb) std::memcpy(J.h_up, c->block_cfg, J.nb);
  std::memcpy(J.h_up + al256(J.nb + 16), J.h_wq, sizeof J.h_wq);
  HIPCK(hipMemcpyAsync(J.dbcfg, J.h_up, al256(J.nb + 16) + sizeof J.h_wq, hipMemcpyHostToDevice,
                       st));
  const Lattice al = anchor_lattice(J.g, c->anchor_log2);
  Lo.n_anchor = al.total;
  HIPCK(launch_anchors<T>(J.g, al, J.X, J.W, J.code, J.anc, c->radius, 0, st));
  const int rc = run_levels<T>(ctx, d, c, J.g, e, J.X, J.W, J.code, J.dbcfg,
                               c->block_log2 ? c->block_cfg : nullptr, J.dwq, J.h_wq, 0, st,
                               J.fast ? c->block_log2 : 0);
  if (rc) return rc;
  HIPCK(hipMemsetAsync(J.hist, 0, (size_t)J.nsym * 4, st));
  if (J.fast) {
    // faces, then block interiors with the brick histogram fused in
    uint32_t lo = c->radius > kBlockHistWin / 2 ? c->radius - kBlockHistWin / 2 : 0;
    if (lo + kBlockHistWin > J.nsym)
      lo = J.nsym > (uint32_t)kBlockHistWin ? J.nsym - kBlockHistWin : 0;
    J.lo = lo;
  } else {
    Span sp(ctx, "histogram", J.N * 2, st);
    HIPCK(launch_histogram(J.code, J.N, J.hist, J.nsym, c->radius, st));
  }
  return HPEZ_OK;
}

template <typename T>
BlockJobHost<T> c_block_job(const CJob<T>& J)
{
  BlockJobHost<T> B;
  B.c = J.c;
  B.g = J.g;
  B.e = J.Lo.e;
  B.X = J.X;
  B.xface = J.xface;
  B.Wg = J.W;
  B.code = J.code;
  B.d_bcfg = J.dbcfg;
  B.h_wq = J.h_wq;
  B.hist = J.hist;
  B.hist_lo = J.lo;
  B.area = J.area;
  B.out = nullptr;
  B.dtype = J.d->dtype;
  return B;
}

// histogram and codebook (Sec. 4 step 4), on the host after the histogram sync
template <typename T>
void c_codebook(CJob<T>& J)
{
  const uint32_t nsym = J.nsym;
  Layout& Lo = J.Lo;
  int rc = huffman_lengths(J.h_hist, nsym, J.h_len);
  if (rc) {
    J.rc = rc;
    return;
  }
  for (uint32_t k = 0; k < nsym; k++)
    if (J.h_len[k]) { Lo.sym_min = k; break; }
  for (uint32_t k = nsym; k-- > 0;)
    if (J.h_len[k]) { Lo.sym_max = k; break; }
  uint64_t bits = 0;
  J.maxlen = 0;
  if (Lo.sym_max >= Lo.sym_min) {
    canonical_codes_range(J.h_len, Lo.sym_min, Lo.sym_max + 1, J.h_cw);
    for_used(J.h_len, Lo.sym_min, Lo.sym_max + 1, [&](uint32_t k) {
      bits += (uint64_t)J.h_hist[k] * J.h_len[k];
      J.maxlen = std::max<uint32_t>(J.maxlen, J.h_len[k]);
    });
  }
  Lo.n_unpred = J.h_hist[0];
  Lo.n_chunks = J.nch;
  Lo.payload_bits = bits;
  layout(&Lo, sizeof(T));
  if (Lo.total > J.cap) {
    J.rc = HPEZ_ENOSPC;
    return;
  }
  write_header(J.h_hdr, J.d, J.c, Lo);
}

// Verbatim values (Sec. 4: unpredictable points) into their section while the
// host builds the codebook: the section's offset depends only on the block
// configurations and anchors.  Needs room for every point to be verbatim (the
// count is known only after the histogram); the rest of the stream, padding
// included, is zeroed around it.
template <typename T>
int c_gather_early(hpez_ctx* ctx, CJob<T>& J, hipStream_t st)
{
  const uint64_t s = sizeof(T);
  Layout t = J.Lo;
  t.n_unpred = t.n_outlier = t.n_patch = t.n_chunks = t.payload_bits = 0;
  t.sym_min = 1;
  t.sym_max = 0;
  layout(&t, s);
  if (J.cap < t.off_unpred + J.N * s) return HPEZ_OK;
  J.early = true;
  J.off_unpred = t.off_unpred;
  HIPCK(hipMemsetAsync(J.out, 0, t.off_unpred, st));
  Span sp(ctx, "gather_unpred", J.N * 2, st);
  HIPCK(launch_gather_unpred<T>(J.code, J.N, J.c->chunk, J.czero, J.zoff, J.tmp2, J.X,
                                (T*)(J.out + t.off_unpred), J.g, st));
  return HPEZ_OK;
}

// assemble the stream
template <typename T>
int c_encode(hpez_ctx* ctx, CJob<T>& J, hipStream_t st)
{
  const Layout& Lo = J.Lo;
  const hpez_config* c = J.c;
  const uint64_t s = sizeof(T);
  uint8_t* out = J.out;
  // codewords above 26 bits go to a long table after the packed one
  uint32_t nlong = 0;
  if (J.maxlen > 26)
    for_used(J.h_len, Lo.sym_min, Lo.sym_max + 1, [&](uint32_t k) { nlong += J.h_len[k] > 26; });
  const uint64_t ntab = Lo.sym_max >= Lo.sym_min ? Lo.sym_max - Lo.sym_min + 1 : 0;
  const uint64_t loff = (ntab + 1) & ~1ull;  // words, 8-byte aligned
  if (loff + 2 * (uint64_t)nlong > J.nsym) {
    // no room for the long table: the encoder's unpacked path reads the full
    // length and codeword tables
    for (uint32_t k = 0; k < J.nsym; k++)
      if (k < Lo.sym_min || k > Lo.sym_max) J.h_cw[k] = 0;
    HIPCK(hipMemcpyAsync(J.dlen, J.h_len, J.nsym, hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(J.dcw, J.h_cw, (size_t)J.nsym * 4, hipMemcpyHostToDevice, st));
  }
  if (J.early && loff + 2 * (uint64_t)nlong <= J.nsym && ((uintptr_t)out & 7) == 0 &&
      Lo.sym_max >= Lo.sym_min) {
    // the small sections, the zero fill after the verbatim values and the
    // encoder's flags in one upload and one launch
    if (Lo.off_unpred != J.off_unpred) return HPEZ_EINVAL;
    const uint64_t vend = Lo.off_unpred + Lo.n_unpred * s;
    const uint64_t nlen = Lo.sym_max - Lo.sym_min + 1;
    const uint64_t a0 = Lo.off_anchor;               // header + block configurations, padded
    const uint64_t a1 = Lo.off_chunks - Lo.off_len;  // code lengths, padded
    uint8_t* h = J.h_stage;
    std::memset(h, 0, a0 + a1);
    std::memcpy(h, J.h_hdr, kHdrBytes);
    if (J.nb) std::memcpy(h + kHdrBytes, c->block_cfg, J.nb);
    std::memcpy(h + a0, J.h_len + Lo.sym_min, nlen);
    uint32_t* tab = reinterpret_cast<uint32_t*>(h + a0 + a1);
    uint64_t* lt = reinterpret_cast<uint64_t*>(tab + loff);
    std::memset(tab, 0, loff * 4);
    uint32_t il = 0;
    for_used(J.h_len, Lo.sym_min, Lo.sym_max + 1, [&](uint32_t sy) {
      if (J.h_len[sy] <= 26) {
        tab[sy - Lo.sym_min] = J.h_cw[sy] << 6 | J.h_len[sy];
      } else {
        lt[il] = (uint64_t)J.h_cw[sy] << 6 | J.h_len[sy];
        tab[sy - Lo.sym_min] = il++ << 6 | 63u;
      }
    });
    HIPCK(hipMemcpyAsync(J.d_stage, h, a0 + a1 + (loff + 2 * (uint64_t)nlong) * 4,
                         hipMemcpyHostToDevice, st));
    const uint64_t vz = (vend + 7) & ~7ull;
    ByteSegs sg;
    std::memset(&sg, 0, sizeof sg);
    auto add = [&](uint8_t* dst, const uint8_t* src, uint64_t n) {
      if (n) sg.s[sg.count++] = ByteSeg{dst, src, n};
    };
    add(out, J.d_stage, a0);
    add(out + Lo.off_anchor, reinterpret_cast<const uint8_t*>(J.anc), Lo.n_anchor * s);
    add(out + vend, nullptr, (vz < Lo.off_len ? vz : Lo.off_len) - vend);
    if (vz < Lo.off_len) add(out + vz, nullptr, Lo.off_len - vz);
    add(out + Lo.off_len, J.d_stage + a0, a1);
    add(out + Lo.off_chunks, nullptr, Lo.total - Lo.off_chunks);
    add(reinterpret_cast<uint8_t*>(J.boff), nullptr, J.nch * 8);
    add(reinterpret_cast<uint8_t*>(J.ticket), nullptr, 4);
    HIPCK(launch_byte_segs(sg, st));
    return encode_payload_packed(ctx, J.code, J.N, c->chunk, Lo.sym_min, Lo.sym_max,
                                 reinterpret_cast<const uint32_t*>(J.d_stage + a0 + a1),
                                 nlong ? reinterpret_cast<const uint64_t*>(J.d_stage + a0 + a1 +
                                                                           loff * 4)
                                       : nullptr,
                                 J.boff, J.ticket, (uint32_t*)(out + Lo.off_payload),
                                 (uint16_t*)(out + Lo.off_chunks), st);
  }
  if (J.early) {
    if (Lo.off_unpred != J.off_unpred) return HPEZ_EINVAL;
    const uint64_t vend = Lo.off_unpred + Lo.n_unpred * s;
    HIPCK(hipMemsetAsync(out + vend, 0, Lo.total - vend, st));
  } else {
    HIPCK(hipMemsetAsync(out, 0, Lo.total, st));
  }
  HIPCK(hipMemcpyAsync(out, J.h_hdr, kHdrBytes, hipMemcpyHostToDevice, st));
  if (J.nb)
    HIPCK(hipMemcpyAsync(out + Lo.off_blocks, c->block_cfg, J.nb, hipMemcpyHostToDevice, st));
  HIPCK(hipMemcpyAsync(out + Lo.off_anchor, J.anc, Lo.n_anchor * s, hipMemcpyDeviceToDevice, st));
  if (Lo.sym_max >= Lo.sym_min)
    HIPCK(hipMemcpyAsync(out + Lo.off_len, J.h_len + Lo.sym_min, Lo.sym_max - Lo.sym_min + 1,
                         hipMemcpyHostToDevice, st));
  if (Lo.n_unpred && !J.early) {
    // verbatim values in stream order (Sec. 4: unpredictable points)
    Span sp(ctx, "gather_unpred", J.N * 2 + Lo.n_unpred * s * 2, st);
    HIPCK(launch_gather_unpred<T>(J.code, J.N, c->chunk, J.czero, J.zoff, J.tmp2, J.X,
                                  (T*)(out + Lo.off_unpred), J.g, st));
  }
  return encode_payload(ctx, J.code, J.N, c->chunk, J.h_len, J.h_cw, Lo.sym_min, Lo.sym_max,
                        J.dlen, J.dcw, J.hist, J.nsym, J.boff, J.ticket, J.h_tab,
                        (uint32_t*)(out + Lo.off_payload), (uint16_t*)(out + Lo.off_chunks), st);
}

// Compress jobs [0, n) of one dtype.  A job's own failure (non-finite input,
// ENOSPC, ...) stays in its rc; device errors end the whole call.
template <typename T>
int compress_jobs(hpez_ctx* ctx, std::vector<CJob<T>>& jobs, hipStream_t st)
{
  const int n = (int)jobs.size();
  if (!n) return HPEZ_OK;
  size_t dev = 0, pin = 0;
  int nfast = 0;
  for (auto& J : jobs) {
    c_init(J);
    dev += c_dev_bytes(J);
    pin += c_pin_bytes(J);
    nfast += J.fast;
  }
  dev += al256(block_tables_bound<T>(nfast > 0 ? nfast : 1)) + 256;
  int rc = ensure_ws(ctx, dev);
  if (rc) return rc;
  rc = ensure_pinned(ctx, pin);
  if (rc) return rc;
  Bump bw{(uint8_t*)ctx->ws};
  Bump pb{ctx->pinned};
  for (auto& J : jobs) c_take(J, bw, pb);

  // the per-field phases of several fields on the context's stream pool (the
  // fields' launches are small and independent)
  hipStream_t ps[hpez_ctx::kPool];
  int np = ctx_fork_pool(ctx, st, n, ps);
  if (np < 0) return HPEZ_EDEVICE;
  auto js = [&](int i) { return np ? ps[i % np] : st; };
  for (int i = 0; i < n; i++) {
    rc = c_minmax(ctx, jobs[i], js(i));
    if (rc) return rc;
  }
  if (np && (rc = ctx_join_pool(ctx, st, np))) return rc;
  HIPCK(hipStreamSynchronize(st));
  std::vector<BlockJobHost<T>> bj;
  np = ctx_fork_pool(ctx, st, n, ps);
  if (np < 0) return HPEZ_EDEVICE;
  for (int i = 0; i < n; i++) {
    CJob<T>& J = jobs[i];
    rc = c_predict(ctx, J, js(i));
    if (rc) return rc;
    if (!J.rc && !J.kind && J.fast) bj.push_back(c_block_job(J));
  }
  if (np && (rc = ctx_join_pool(ctx, st, np))) return rc;
  rc = block_phase<T>(ctx, bj, 0, bw, st);
  if (rc) return rc;
  for (auto& J : jobs)
    if (!J.rc && !J.kind)
      HIPCK(hipMemcpyAsync(J.h_hist, J.hist, (size_t)J.nsym * 4, hipMemcpyDeviceToHost, st));
  // the histograms are on the host once ev_sync completes; the verbatim values
  // are gathered meanwhile
  if (!ctx->ev_sync) HIPCK(hipEventCreateWithFlags(&ctx->ev_sync, hipEventDisableTiming));
  HIPCK(hipEventRecord(ctx->ev_sync, st));
  for (auto& J : jobs)
    if (!J.rc && !J.kind && (rc = c_gather_early(ctx, J, st))) return rc;
  HIPCK(hipEventSynchronize(ctx->ev_sync));
  host_parallel(n, [&](int i) {
    if (!jobs[i].rc && !jobs[i].kind) c_codebook(jobs[i]);
  });
  np = ctx_fork_pool(ctx, st, n, ps);
  if (np < 0) return HPEZ_EDEVICE;
  for (int i = 0; i < n; i++) {
    CJob<T>& J = jobs[i];
    if (J.rc || J.kind) continue;
    rc = c_encode(ctx, J, js(i));
    if (rc) return rc;
  }
  if (np && (rc = ctx_join_pool(ctx, st, np))) return rc;
  HIPCK(hipStreamSynchronize(st));
  prof_collect(ctx);
  // the Lorenzo alternative (Sec. 6.5) runs per field after the rest
  for (auto& J : jobs) {
    if (J.rc || J.kind != 2) continue;
    uint64_t sz = 0;
    J.rc = lorenzo_compress<T>(ctx, J.d, J.X, J.c, J.Lo.e, J.out, J.cap, &sz, st);
    if (J.rc == HPEZ_EDEVICE) return J.rc;
    J.Lo.total = sz;
  }
  return HPEZ_OK;
}

// ---------------------------------------------------------------------------
// Decompression of one stream as a job in phases: header; code lengths and
// block configurations; decode, verbatim values, anchors, levels; status.
template <typename T>
struct DJob {
  const uint8_t* in = nullptr;
  T* out = nullptr;
  hpez_field_desc d;
  hpez_config c;
  Layout Lo;
  int rc = HPEZ_OK;
  uint64_t N = 0, nb = 0, nch = 0;
  uint32_t nsym = 0;
  Geom g;
  bool fast = false;
  double h_wq[3 * 16 * 4];
  DecodeArgs da;
  uint32_t nused = 0;  // symbols with a code
  // the first bytes of the stream (host copy), or null
  const uint8_t* h_prefix = nullptr;
  uint64_t prefix_len = 0;
  // device workspace
  uint16_t* code = nullptr;
  uint32_t* czero = nullptr;
  uint64_t* zoff = nullptr;
  uint64_t* tmp2 = nullptr;
  // one region uploaded at once (dtabs): status, MD weights, first-level
  // table, second-level tables, sorted symbols
  uint8_t* dtabs = nullptr;
  uint64_t tabs_len = 0;
  uint64_t* tflags = nullptr;  // the decoder's look-back flags (in dtabs, zeroed)
  bool fcode2 = false;  // the decoder wrote family 2's codes to the face code array
  double* dwq = nullptr;
  uint32_t* dlut = nullptr;
  uint16_t* dsorted = nullptr;
  uint32_t* dsub = nullptr;
  int* status = nullptr;
  long long* lv = nullptr;
  void* area = nullptr;
  // pinned host staging
  uint8_t* h_len = nullptr;
  uint8_t* h_bcfg = nullptr;
  int* h_status = nullptr;
  uint64_t* h_tot = nullptr;
  uint32_t* h_lut = nullptr;
  uint16_t* h_sorted = nullptr;
  uint32_t* h_sub = nullptr;
  uint8_t* h_tabs = nullptr;  // host image of dtabs
};

// offsets in the decode table region
constexpr uint64_t kTabWq = 16, kTabLut = kTabWq + 3 * 16 * 4 * 8,
                   kTabSub = kTabLut + ((uint64_t)4 << kLutBits);
template <typename T>
uint64_t d_tabs_bytes(const DJob<T>& J)
{
  return kTabSub + (uint64_t)kDecSub * 4 + (uint64_t)J.nsym * 2 + 16 + ((J.nch + 255) / 256) * 8;
}

template <typename T>
void d_init(DJob<T>& J)
{
  J.N = points_of(&J.d);
  J.nsym = 2 * J.c.radius;
  J.nb = J.Lo.n_blocks;
  J.nch = J.Lo.n_chunks;
  J.g = make_geom(&J.d, J.c.frozen_dim);
  J.fast = J.Lo.predictor == HPEZ_INTERP && block_fast_ok<T>(&J.c, J.g);
}

template <typename T>
size_t d_dev_bytes(const DJob<T>& J)
{
  size_t b = al256(J.N * 2) + al256((J.nch + 1) * 4) + 2 * al256((J.nch + 1) * 8) +
             al256(d_tabs_bytes(J));
  if (J.Lo.predictor == 1) b += al256(J.N * 8);
  if (J.fast) b += al256(block_fast_bytes<T>(J.g));
  return b + 256;
}

template <typename T>
size_t d_pin_bytes(const DJob<T>& J)
{
  return al256(J.nsym) + al256(J.nb) + al256(16) + al256(16) + al256(J.nsym * 2) +
         al256(d_tabs_bytes(J)) + 256;
}

template <typename T>
void d_take(DJob<T>& J, Bump& bw, Bump& pb)
{
  J.code = bw.take<uint16_t>(J.N);
  J.czero = bw.take<uint32_t>(J.nch + 1);
  J.zoff = bw.take<uint64_t>(J.nch + 1);
  J.tmp2 = bw.take<uint64_t>(J.nch + 1);
  J.dtabs = bw.take<uint8_t>(d_tabs_bytes(J));
  J.status = reinterpret_cast<int*>(J.dtabs);
  J.dwq = reinterpret_cast<double*>(J.dtabs + kTabWq);
  J.dlut = reinterpret_cast<uint32_t*>(J.dtabs + kTabLut);
  J.dsub = reinterpret_cast<uint32_t*>(J.dtabs + kTabSub);
  J.dsorted = nullptr;  // placed after the used second-level entries (d_tables)
  if (J.Lo.predictor == 1) J.lv = bw.take<long long>(J.N);
  if (J.fast) J.area = bw.take<uint8_t>(block_fast_bytes<T>(J.g));
  J.h_len = pb.take<uint8_t>(J.nsym);
  J.h_bcfg = pb.take<uint8_t>(J.nb);
  J.h_status = pb.take<int>(4);
  J.h_tot = pb.take<uint64_t>(2);
  J.h_tabs = pb.take<uint8_t>(d_tabs_bytes(J));
  J.h_lut = reinterpret_cast<uint32_t*>(J.h_tabs + kTabLut);
  J.h_sub = reinterpret_cast<uint32_t*>(J.h_tabs + kTabSub);
  J.h_sorted = pb.take<uint16_t>(J.nsym);
}

// constant field, or the copies of code lengths and block configurations
// (from the host prefix of the stream when they lie in it; *dev is set when a
// device copy was needed)
template <typename T>
int d_fetch(DJob<T>& J, hipStream_t st, bool* dev)
{
  const Layout& Lo = J.Lo;
  const uint64_t s = sizeof(T);
  if (Lo.predictor == 2) {
    // constant field: broadcast by doubling copies
    HIPCK(hipMemcpyAsync(J.out, J.in + Lo.off_anchor, s, hipMemcpyDeviceToDevice, st));
    uint64_t have = 1;
    while (have < J.N) {
      const uint64_t m = have < J.N - have ? have : J.N - have;
      HIPCK(hipMemcpyAsync(J.out + have, J.out, m * s, hipMemcpyDeviceToDevice, st));
      have += m;
    }
    return HPEZ_OK;
  }
  std::memset(J.h_len, 0, J.nsym);
  auto fetch = [&](void* dst, uint64_t off, uint64_t bytes) -> int {
    if (!bytes) return HPEZ_OK;
    if (J.h_prefix && off + bytes <= J.prefix_len) {
      std::memcpy(dst, J.h_prefix + off, bytes);
      return HPEZ_OK;
    }
    *dev = true;
    HIPCK(hipMemcpyAsync(dst, J.in + off, bytes, hipMemcpyDeviceToHost, st));
    return HPEZ_OK;
  };
  int rc = HPEZ_OK;
  if (Lo.sym_max >= Lo.sym_min)
    rc = fetch(J.h_len + Lo.sym_min, Lo.off_len, Lo.sym_max - Lo.sym_min + 1);
  if (!rc && J.nb) rc = fetch(J.h_bcfg, Lo.off_blocks, J.nb);
  return rc;
}

// host: validate lengths and block configurations, build the decode tables
template <typename T>
void d_tables(DJob<T>& J)
{
  const uint32_t nsym = J.nsym;
  for (uint64_t b = 0; b < J.nb; b++)
    if (J.h_bcfg[b] >= J.c.n_cand) {
      J.rc = HPEZ_ECORRUPT;
      return;
    }
  uint64_t kraft = 0, used = 0;
  const uint32_t lo = J.Lo.sym_max >= J.Lo.sym_min ? J.Lo.sym_min : 0;
  const uint32_t hi = J.Lo.sym_max >= J.Lo.sym_min ? J.Lo.sym_max + 1 : 0;
  (void)nsym;
  bool too_long = false;
  for_used(J.h_len, lo, hi, [&](uint32_t k) {
    if (J.h_len[k] > kLmax) {
      too_long = true;
      return;
    }
    kraft += 1ull << (kLmax - J.h_len[k]);
    used++;
  });
  if (too_long) {
    J.rc = HPEZ_ECORRUPT;
    return;
  }
  if (J.N > 0 && !(kraft == (1ull << kLmax) || (used == 1 && kraft == (1ull << (kLmax - 1))))) {
    J.rc = HPEZ_ECORRUPT;
    return;
  }
  DecodeArgs& da = J.da;
  std::memset(&da, 0, sizeof da);
  da.n = J.N;
  da.nch = J.nch;
  da.nbits = J.Lo.payload_bits;
  da.chunk = J.c.chunk;
  decode_tables_range(J.h_len, lo, hi, J.h_lut, J.h_sorted, da.lim, da.base);
  uint32_t nshort = 0, nused = 0;
  for_used(J.h_len, lo, hi, [&](uint32_t k) {
    nused++;
    nshort += J.h_len[k] <= kLutBits;
  });
  J.nused = nused;
  da.long_first = nshort;
  da.n_long = nused - nshort;
  // long codes by second-level tables when they fit (the first level is updated)
  da.n_sub = da.n_long ? decode_subtables(J.h_len, lo, hi, J.h_lut, J.h_sub, kDecSub) : 0;
  md_table(&J.c, J.h_wq);
  // the region's image: status 0, weights, tables, then the sorted symbols
  std::memset(J.h_tabs, 0, kTabWq);
  std::memcpy(J.h_tabs + kTabWq, J.h_wq, sizeof J.h_wq);
  const uint64_t so = kTabSub + (uint64_t)da.n_sub * 4;
  std::memcpy(J.h_tabs + so, J.h_sorted, (size_t)J.nused * 2);
  J.dsorted = reinterpret_cast<uint16_t*>(J.dtabs + so);
  const uint64_t fo = (so + (uint64_t)J.nused * 2 + 7) & ~7ull;
  const uint64_t nfl = (J.nch + 255) / 256;
  std::memset(J.h_tabs + fo, 0, nfl * 8);
  J.tflags = reinterpret_cast<uint64_t*>(J.dtabs + fo);
  J.tabs_len = fo + nfl * 8;
}

// decode, verbatim values, anchors and the levels down to the block phase
template <typename T>
int d_decode(hpez_ctx* ctx, DJob<T>& J, hipStream_t st)
{
  const Layout& Lo = J.Lo;
  const hpez_config* c = &J.c;
  const uint8_t* in = J.in;
  const uint64_t N = J.N, nch = J.nch;
  const uint64_t s = sizeof(T);
  HIPCK(hipMemcpyAsync(J.dtabs, J.h_tabs, J.tabs_len, hipMemcpyHostToDevice, st));
  // every brick full and one chunk per brick slab: the decoder also writes the
  // codes of the face planes x2 = 0 (mod 32) to family 2's compact code array
  J.da.f2code = nullptr;
  const int64_t Bk = (int64_t)1 << kBrickLog2;
  if (J.fast && J.c.chunk == 1024 && Bk == 32 && J.g.n[3] == 1 && J.g.act[2] &&
      J.g.n[0] % Bk == 0 && J.g.n[1] % Bk == 0 && J.g.n[2] % Bk == 0) {
    const FaceGeo f = block_face_arrays<T>(J.g, J.area);
    J.da.f2code = f.code[2];
    J.da.f2_plane = (uint64_t)f.plane[2];
    J.da.f2_n1 = (uint32_t)J.g.n[1];
    J.da.nbk1 = (uint32_t)(J.g.n[1] / Bk);
    J.da.nbk2 = (uint32_t)(J.g.n[2] / Bk);
    J.fcode2 = true;
  }
  {
    Span sp(ctx, "decode", N * 2 + (Lo.payload_bits + 7) / 8, st);
    HIPCK(launch_decode2(J.da, (const uint32_t*)(in + Lo.off_payload),
                         (const uint16_t*)(in + Lo.off_chunks), J.tflags, J.dlut, J.dsorted,
                         J.dsub, J.code, J.czero, J.status, st));
  }
  HIPCK(launch_scan_u32_to_u64(J.czero, nch, J.zoff, J.zoff + nch, J.tmp2, st));
  if (Lo.predictor == 1) {
    // Lorenzo alternative: residuals, running sums, patches
    const Geom gl = make_geom(&J.d, -1);
    Span sp(ctx, "lorenzo_rebuild", N * (2 + s), st);
    HIPCK(launch_lorenzo_rebuild<T>(J.code, gl, N, c->radius, c->chunk, J.czero, J.zoff,
                                    (const long long*)(in + Lo.off_outl), Lo.n_outlier,
                                    (const uint64_t*)(in + Lo.off_pidx),
                                    (const T*)(in + Lo.off_pval), Lo.n_patch, 2.0 * Lo.e, J.lv,
                                    J.out, J.status, st));
    return HPEZ_OK;
  }
  if (Lo.n_unpred)
    HIPCK(launch_scatter_unpred2<T>(J.code, N, c->chunk, J.czero, J.zoff,
                                    (const T*)(in + Lo.off_unpred), Lo.n_unpred, J.out, J.status,
                                    J.g, st));
  const Lattice al = anchor_lattice(J.g, c->anchor_log2);
  if (al.total != Lo.n_anchor) {
    J.rc = HPEZ_ECORRUPT;
    return HPEZ_OK;
  }
  HIPCK(launch_anchors<T>(J.g, al, nullptr, J.out, J.code, (T*)(in + Lo.off_anchor), c->radius, 1,
                          st));
  return run_levels<T>(ctx, &J.d, c, J.g, Lo.e, nullptr, J.out, J.code, in + Lo.off_blocks,
                       J.nb ? J.h_bcfg : nullptr, J.dwq, J.h_wq, 1, st,
                       J.fast ? c->block_log2 : 0);
}

template <typename T>
BlockJobHost<T> d_block_job(const DJob<T>& J)
{
  BlockJobHost<T> B;
  B.c = &J.c;
  B.g = J.g;
  B.e = J.Lo.e;
  B.X = nullptr;
  B.Wg = J.out;
  B.code = J.code;
  B.d_bcfg = J.in + J.Lo.off_blocks;
  B.h_wq = J.h_wq;
  B.hist = nullptr;
  B.hist_lo = 0;
  B.area = J.area;
  B.fcode2 = J.fcode2;
  B.out = J.out;
  B.dtype = J.d.dtype;
  return B;
}

// Decompress jobs [0, n) of one dtype whose headers are read (d, c, Lo).
template <typename T>
int decompress_jobs(hpez_ctx* ctx, std::vector<DJob<T>>& jobs, hipStream_t st)
{
  const int n = (int)jobs.size();
  if (!n) return HPEZ_OK;
  size_t dev = 0, pin = 0;
  int nfast = 0;
  for (auto& J : jobs) {
    d_init(J);
    dev += d_dev_bytes(J);
    pin += d_pin_bytes(J);
    nfast += J.fast;
  }
  dev += al256(block_tables_bound<T>(nfast > 0 ? nfast : 1)) + 256;
  int rc = ensure_ws(ctx, dev);
  if (rc) return rc;
  rc = ensure_pinned(ctx, pin);
  if (rc) return rc;
  Bump bw{(uint8_t*)ctx->ws};
  Bump pb{ctx->pinned};
  for (auto& J : jobs) d_take(J, bw, pb);
  bool need_sync = false;
  for (auto& J : jobs) {
    // a recording keeps the lengths and configurations the eager call fetched
    // (same staging addresses); constant fields still record their copies
    if (ctx->capture && J.Lo.predictor != 2) continue;
    rc = d_fetch(J, st, &need_sync);
    if (rc) return rc;
  }
  if (need_sync) HIPCK(hipStreamSynchronize(st));
  host_parallel(n, [&](int i) {
    if (jobs[i].Lo.predictor != 2) d_tables(jobs[i]);
  });
  std::vector<BlockJobHost<T>> bj;
  // decode, verbatim values, anchors and the levels above the blocks of
  // several fields on the context's stream pool
  int nd = 0;
  for (auto& J : jobs) nd += !J.rc && J.Lo.predictor != 2;
  hipStream_t ps[hpez_ctx::kPool];
  const int np = ctx_fork_pool(ctx, st, nd, ps);
  if (np < 0) return HPEZ_EDEVICE;
  int k = 0;
  for (auto& J : jobs) {
    if (J.rc || J.Lo.predictor == 2) continue;
    rc = d_decode(ctx, J, np ? ps[k++ % np] : st);
    if (rc) return rc;
    if (!J.rc && J.fast && J.Lo.predictor == HPEZ_INTERP) bj.push_back(d_block_job(J));
  }
  if (np && (rc = ctx_join_pool(ctx, st, np))) return rc;
  rc = block_phase<T>(ctx, bj, 1, bw, st);
  if (rc) return rc;
  if (ctx->capture) return HPEZ_OK;  // checks: decompress_group
  for (auto& J : jobs) {
    if (J.rc || J.Lo.predictor == 2) continue;
    HIPCK(hipMemcpyAsync(J.h_status, J.status, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCK(hipMemcpyAsync(J.h_tot, J.zoff + J.nch, 8, hipMemcpyDeviceToHost, st));
  }
  HIPCK(hipStreamSynchronize(st));
  prof_collect(ctx);
  for (auto& J : jobs) {
    if (J.rc || J.Lo.predictor == 2) continue;
    const uint64_t want = J.Lo.predictor == 1 ? J.Lo.n_outlier : J.Lo.n_unpred;
    if (*J.h_status || J.h_tot[0] != want) J.rc = HPEZ_ECORRUPT;
  }
  return HPEZ_OK;
}

// device bytes of one compress (op 0) or decompress (op 1) job, block tables included
template <typename T>
uint64_t job_footprint(const hpez_field_desc* d, const hpez_config* c, int op)
{
  const uint64_t extra = al256(block_tables_bound<T>(1)) + 256;
  if (op == 0) {
    CJob<T> J;
    J.d = d;
    J.c = c;
    c_init(J);
    return c_dev_bytes(J) + extra;
  }
  DJob<T> J;
  J.d = *d;
  J.c = *c;
  std::memset(&J.Lo, 0, sizeof J.Lo);
  J.Lo.predictor = c->predictor;
  J.Lo.n_blocks = n_blocks(d, c);
  J.Lo.n_chunks = (points_of(d) + c->chunk - 1) / c->chunk;
  d_init(J);
  return d_dev_bytes(J) + extra;
}

}  // namespace

namespace {
// Integer fields of a batch: their values as float64 in the context's
// auxiliary buffer; in[i] is redirected there.
int int_inputs(hpez_ctx* ctx, int n, const hpez_field_desc* d, const void** in, hipStream_t st)
{
  size_t aux = 0;
  for (int i = 0; i < n; i++)
    if (dtype_int(d[i].dtype)) aux += al256(points_of(&d[i]) * 8);
  if (!aux) return HPEZ_OK;
  int rc = HPEZ_OK;
  uint8_t* p = (uint8_t*)ctx_aux(ctx, aux, &rc);
  if (rc) return rc;
  for (int i = 0; i < n; i++) {
    if (!dtype_int(d[i].dtype)) continue;
    const uint64_t N = points_of(&d[i]);
    if (launch_int_to_f64(in[i], d[i].dtype, (double*)p, N, st) != hipSuccess) return HPEZ_EDEVICE;
    in[i] = p;
    p += al256(N * 8);
  }
  return HPEZ_OK;
}

template <typename T>
int compress_group(hpez_ctx* ctx, int n, const hpez_field_desc* d, const void* const* d_in,
                   const hpez_config* c, void* const* d_out, const uint64_t* out_cap,
                   uint64_t* out_sizes, const std::vector<int>& idx, int* first_rc,
                   hipStream_t st)
{
  (void)n;
  std::vector<CJob<T>> jobs(idx.size());
  for (size_t k = 0; k < idx.size(); k++) {
    const int i = idx[k];
    jobs[k].d = &d[i];
    jobs[k].X = (const T*)d_in[i];
    jobs[k].c = &c[i];
    jobs[k].out = (uint8_t*)d_out[i];
    jobs[k].cap = out_cap[i];
  }
  const int rc = compress_jobs<T>(ctx, jobs, st);
  if (rc) return rc;
  for (size_t k = 0; k < idx.size(); k++) {
    const int i = idx[k];
    out_sizes[i] = jobs[k].rc ? 0 : jobs[k].Lo.total;
    if (jobs[k].rc && !*first_rc) *first_rc = jobs[k].rc;
  }
  return HPEZ_OK;
}

template <typename T>
int decompress_group(hpez_ctx* ctx, std::vector<DJob<T>>& jobs, const std::vector<int>& idx,
                     int* rcs, hipStream_t st)
{
  const int rc = decompress_jobs<T>(ctx, jobs, st);
  if (rc) return rc;
  for (size_t k = 0; k < idx.size(); k++) {
    rcs[idx[k]] = jobs[k].rc;
    const DJob<T>& J = jobs[k];
    if (ctx->capture && !J.rc && J.Lo.predictor != 2)
      ctx->checks.push_back({idx[k], J.status, J.zoff + J.nch,
                             J.Lo.predictor == 1 ? J.Lo.n_outlier : J.Lo.n_unpred});
  }
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
  if (ctx->aux) (void)hipFree(ctx->aux);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->pin_tab) (void)hipHostFree(ctx->pin_tab);
  if (ctx->pin_pre) (void)hipHostFree(ctx->pin_pre);
  if (ctx->ev_sync) (void)hipEventDestroy(ctx->ev_sync);
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  for (int i = 0; i < ctx->pool_n; i++) {
    (void)hipEventDestroy(ctx->pool_join[i]);
    (void)hipStreamDestroy(ctx->pool[i]);
  }
  if (ctx->pool_fork) (void)hipEventDestroy(ctx->pool_fork);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  delete ctx;
}

int hpez_ctx_trim(hpez_ctx* ctx, uint64_t keep_bytes)
{
  if (!ctx) return HPEZ_EINVAL;
  DevScope ds(ctx->device);
  if (ctx->ws && ctx->ws_bytes > keep_bytes) {
    if (hipFree(ctx->ws) != hipSuccess) return HPEZ_EDEVICE;
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  if (ctx->aux && ctx->aux_bytes > keep_bytes) {
    if (hipFree(ctx->aux) != hipSuccess) return HPEZ_EDEVICE;
    ctx->aux = nullptr;
    ctx->aux_bytes = 0;
  }
  if (ctx->pinned && ctx->pinned_bytes > keep_bytes) {
    (void)hipHostFree(ctx->pinned);
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
  }
  return HPEZ_OK;
}

int hpez_ctx_set_limit(hpez_ctx* ctx, uint64_t max_workspace_bytes)
{
  if (!ctx) return HPEZ_EINVAL;
  ctx->ws_limit = (size_t)max_workspace_bytes;
  return HPEZ_OK;
}

int hpez_ctx_workspace(const hpez_ctx* ctx, uint64_t* bytes)
{
  if (!ctx || !bytes) return HPEZ_EINVAL;
  *bytes = ctx->ws_bytes;
  return HPEZ_OK;
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
  if (c->chunk < 64 || c->radius < 1 || c->radius > 32768) return HPEZ_EINVAL;
  const uint64_t N = points_of(d);
  // integer fields: plus their float64 copy (the context's auxiliary buffer)
  const uint64_t aux = dtype_int(d->dtype) ? al256(N * 8) : 0;
  if (op == 2) {
    *bytes = tune_footprint(d, c) + aux;
    return HPEZ_OK;
  }
  hpez_config cc = *c;
  cc.block_cfg = nullptr;
  if (d->dtype == HPEZ_F32) *bytes = job_footprint<float>(d, &cc, op);
  else *bytes = job_footprint<double>(d, &cc, op);
  *bytes += aux;
  return HPEZ_OK;
}

int hpez_compress(hpez_ctx* ctx, const hpez_field_desc* d, const void* d_in,
                  const hpez_config* c, void* d_out, uint64_t out_cap, uint64_t* out_size,
                  hipStream_t stream)
{
  if (!out_size) return HPEZ_EINVAL;
  return hpez_compress_batch(ctx, 1, d, &d_in, c, &d_out, &out_cap, out_size, stream);
}


int hpez_compress_batch(hpez_ctx* ctx, int n, const hpez_field_desc* d,
                        const void* const* d_in, const hpez_config* c, void* const* d_out,
                        const uint64_t* out_cap, uint64_t* out_sizes, hipStream_t stream)
{
  if (!ctx || n < 0 || (n > 0 && (!d || !d_in || !c || !d_out || !out_cap || !out_sizes)))
    return HPEZ_EINVAL;
  for (int i = 0; i < n; i++) {
    if (!d_in[i] || !d_out[i]) return HPEZ_EINVAL;
    int rc = check_desc(&d[i]);
    if (rc) return rc;
    rc = check_cfg(&d[i], &c[i], true);
    if (rc) return rc;
    out_sizes[i] = 0;
  }
  DevScope ds(ctx->device);
  // integer fields: their values as float64 (the method runs in double on them)
  std::vector<const void*> in(d_in, d_in + n);
  int rc = int_inputs(ctx, n, d, in.data(), stream);
  if (rc) return rc;
  std::vector<int> f32, f64;
  for (int i = 0; i < n; i++) (d[i].dtype == HPEZ_F32 ? f32 : f64).push_back(i);
  int first = HPEZ_OK;
  if (!f32.empty())
    rc = compress_group<float>(ctx, n, d, in.data(), c, d_out, out_cap, out_sizes, f32, &first,
                               stream);
  if (!rc && !f64.empty())
    rc = compress_group<double>(ctx, n, d, in.data(), c, d_out, out_cap, out_sizes, f64, &first,
                                stream);
  if (rc) ctx_drain(ctx, stream);
  return rc ? rc : first;
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
  int rc1 = HPEZ_OK;
  const int rc = hpez_decompress_batch(ctx, 1, &d_in, &in_size, &d_out, &out_cap, &rc1, stream);
  return rc ? rc : rc1;
}

int hpez_decompress_batch(hpez_ctx* ctx, int n, const void* const* d_in, const uint64_t* in_size,
                          void* const* d_out, const uint64_t* out_cap, int* rcs,
                          hipStream_t stream)
{
  if (!ctx || n < 0 || (n > 0 && (!d_in || !in_size || !d_out || !out_cap || !rcs)))
    return HPEZ_EINVAL;
  for (int i = 0; i < n; i++)
    if (!d_in[i] || !d_out[i]) return HPEZ_EINVAL;
  if (!n) return HPEZ_OK;
  DevScope ds(ctx->device);
  // every stream's first kPrefixBytes (header, and usually the block
  // configurations and code lengths) in one synchronization
  int rc = ensure_pin_pre(ctx, (size_t)n * kPrefixBytes);
  if (rc) return rc;
  for (int i = 0; i < n; i++) {
    rcs[i] = in_size[i] < (uint64_t)kHdrBytes ? HPEZ_ECORRUPT : HPEZ_OK;
    if (!rcs[i] && !ctx->capture)  // a recording reads the eager call's prefixes
      HIPCK(hipMemcpyAsync(ctx->pin_pre + (size_t)i * kPrefixBytes, d_in[i],
                           std::min<uint64_t>(in_size[i], kPrefixBytes), hipMemcpyDeviceToHost,
                           stream));
  }
  if (!ctx->capture) HIPCK(hipStreamSynchronize(stream));
  std::vector<int> i32, i64;
  std::vector<DJob<float>> j32;
  std::vector<DJob<double>> j64;
  for (int i = 0; i < n; i++) {
    if (rcs[i]) continue;
    hpez_field_desc dd;
    hpez_config cc;
    Layout L;
    int r = read_header(ctx->pin_pre + (size_t)i * kPrefixBytes, in_size[i], &dd, &cc, &L);
    if (!r && L.total > in_size[i]) r = HPEZ_ECORRUPT;
    if (!r && out_cap[i] < points_of(&dd) * dtype_size(dd.dtype)) r = HPEZ_ENOSPC;
    rcs[i] = r;
    if (r) continue;
    if (dd.dtype == HPEZ_F32) {
      j32.emplace_back();
      DJob<float>& J = j32.back();
      J.in = (const uint8_t*)d_in[i];
      J.h_prefix = ctx->pin_pre + (size_t)i * kPrefixBytes;
      J.prefix_len = std::min<uint64_t>(in_size[i], kPrefixBytes);
      J.out = (float*)d_out[i];
      J.d = dd;
      J.c = cc;
      J.Lo = L;
      i32.push_back(i);
    } else {
      j64.emplace_back();
      DJob<double>& J = j64.back();
      J.in = (const uint8_t*)d_in[i];
      J.h_prefix = ctx->pin_pre + (size_t)i * kPrefixBytes;
      J.prefix_len = std::min<uint64_t>(in_size[i], kPrefixBytes);
      J.out = (double*)d_out[i];  // integer fields: set to a float64 buffer below
      J.d = dd;
      J.c = cc;
      J.Lo = L;
      i64.push_back(i);
    }
  }
  // integer streams decode into float64 buffers (aux), then to their type
  size_t aux = 0;
  for (auto& J : j64)
    if (dtype_int(J.d.dtype)) aux += al256(points_of(&J.d) * 8);
  uint8_t* ap = nullptr;
  if (aux) {
    ap = (uint8_t*)ctx_aux(ctx, aux, &rc);
    if (rc) return rc;
  }
  std::vector<void*> int_out(j64.size(), nullptr);
  for (size_t k = 0; k < j64.size(); k++) {
    DJob<double>& J = j64[k];
    if (!dtype_int(J.d.dtype)) continue;
    int_out[k] = (void*)J.out;
    J.out = (double*)ap;
    ap += al256(points_of(&J.d) * 8);
  }
  rc = decompress_group<float>(ctx, j32, i32, rcs, stream);
  if (!rc) rc = decompress_group<double>(ctx, j64, i64, rcs, stream);
  if (rc) {
    ctx_drain(ctx, stream);
    return rc;
  }
  for (size_t k = 0; k < j64.size(); k++) {
    if (!int_out[k] || rcs[i64[k]]) continue;
    HIPCK(launch_f64_to_int(j64[k].out, j64[k].d.dtype, int_out[k], points_of(&j64[k].d), stream));
  }
  if (aux && !ctx->capture) HIPCK(hipStreamSynchronize(stream));
  for (int i = 0; i < n; i++)
    if (rcs[i]) return rcs[i];
  return HPEZ_OK;
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

int hpez_profile_only(hpez_ctx* ctx, const char* group)
{
  if (!ctx) return HPEZ_EINVAL;
  ctx->prof_only = group ? group : "";
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

void* ctx_aux(hpez_ctx* c, size_t bytes, int* rc)
{
  *rc = HPEZ_OK;
  if (c->aux_bytes >= bytes) return c->aux;
  if (c->fixed) {
    *rc = HPEZ_ENOMEM;
    return nullptr;
  }
  if (c->aux) (void)hipFree(c->aux);
  c->aux = nullptr;
  c->aux_bytes = 0;
  if (hipMalloc(&c->aux, bytes) != hipSuccess) {
    c->aux = nullptr;
    *rc = HPEZ_ENOMEM;
    return nullptr;
  }
  c->aux_bytes = bytes;
  return c->aux;
}

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

uint8_t* ctx_pin_tab(hpez_ctx* c, size_t bytes, int* rc)
{
  *rc = ensure_pin_tab(c, bytes);
  return *rc ? nullptr : c->pin_tab;
}

int ctx_device(hpez_ctx* c) { return c->device; }

static uint64_t tile_key(int kind, int dtype, uint64_t work)
{
  int b = 0;
  while (b < 63 && (work >> (b + 1))) b++;  // floor log2
  return (uint64_t)kind << 16 | (uint64_t)dtype << 8 | (uint64_t)b;
}

void ctx_tile_seen(hpez_ctx* c, bool clear, std::vector<uint64_t>* keys)
{
  if (keys) keys->assign(c->tile_seen.begin(), c->tile_seen.end());
  if (clear) c->tile_seen.clear();
}

void ctx_tile_try(hpez_ctx* c, uint64_t key, uint32_t value)
{
  if (value) c->tile_try[key] = value;
  else c->tile_try.erase(key);
}

void ctx_tile_set(hpez_ctx* c, uint64_t key, uint32_t value) { c->tiles[key] = value; }

uint32_t ctx_tile(hpez_ctx* c, int kind, int dtype, uint64_t work, uint32_t deflt)
{
  const uint64_t k = tile_key(kind, dtype, work);
  c->tile_seen.insert(k);
  auto t = c->tile_try.find(k);
  if (t != c->tile_try.end()) return t->second;
  auto f = c->tiles.find(k);
  return f != c->tiles.end() ? f->second : deflt;
}

hipStream_t ctx_fork(hpez_ctx* c, hipStream_t st)
{
  if (c->fixed) return nullptr;  // everything on the caller's stream
  if (!c->side) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
      if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
      c->ev_fork = nullptr;
      (void)hipStreamDestroy(s);
      return nullptr;
    }
    c->side = s;
  }
  if (hipEventRecord(c->ev_fork, st) != hipSuccess ||
      hipStreamWaitEvent(c->side, c->ev_fork, 0) != hipSuccess)
    return nullptr;
  return c->side;
}

int ctx_join(hpez_ctx* c, hipStream_t st)
{
  if (hipEventRecord(c->ev_join, c->side) != hipSuccess ||
      hipStreamWaitEvent(st, c->ev_join, 0) != hipSuccess)
    return HPEZ_EDEVICE;
  return HPEZ_OK;
}

// Up to k streams (at most hpez_ctx::kPool) for independent per-field work,
// each made to wait for the work queued so far on st; returns how many (0:
// keep everything on st, as fixed contexts do), or -1 when a HIP call failed.
// ctx_join_pool makes st wait for all of them.  A recording uses the streams
// the eager call made (the fork and join events make them branches of the
// recorded graph) and creates none.
int ctx_fork_pool(hpez_ctx* c, hipStream_t st, int k, hipStream_t* out)
{
  if ((c->fixed && !c->capture) || k < 2) return 0;
  if (k > hpez_ctx::kPool) k = hpez_ctx::kPool;
  while (!c->capture && c->pool_n < k) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) break;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipStreamDestroy(s);
      break;
    }
    c->pool[c->pool_n] = s;
    c->pool_join[c->pool_n] = e;
    c->pool_n++;
  }
  if (!c->pool_fork && (c->capture || hipEventCreateWithFlags(&c->pool_fork, hipEventDisableTiming) !=
                                         hipSuccess)) {
    c->pool_fork = nullptr;
    return 0;
  }
  if (k > c->pool_n) k = c->pool_n;
  if (k < 2) return 0;
  if (hipEventRecord(c->pool_fork, st) != hipSuccess) return -1;
  for (int i = 0; i < k; i++) {
    if (hipStreamWaitEvent(c->pool[i], c->pool_fork, 0) != hipSuccess) return -1;
    out[i] = c->pool[i];
  }
  return k;
}

int ctx_join_pool(hpez_ctx* c, hipStream_t st, int k)
{
  for (int i = 0; i < k; i++)
    if (hipEventRecord(c->pool_join[i], c->pool[i]) != hipSuccess ||
        hipStreamWaitEvent(st, c->pool_join[i], 0) != hipSuccess)
      return HPEZ_EDEVICE;
  return HPEZ_OK;
}

// After a call fails between its launches (a call-level error other than a
// failed HIP call): wait for the work it queued on the caller's stream, the
// second stream and the pool, so that no copy from the context's host staging
// is still pending when the next call rewrites that staging.  Not while
// recording a plan (nothing runs then).  Errors of the waits are ignored.
void ctx_drain(hpez_ctx* c, hipStream_t st)
{
  if (c->capture) return;
  (void)hipStreamSynchronize(st);
  if (c->side) (void)hipStreamSynchronize(c->side);
  for (int i = 0; i < c->pool_n; i++) (void)hipStreamSynchronize(c->pool[i]);
}

hipEvent_t ctx_span_begin(hpez_ctx* c, hipStream_t st, const char* name)
{
  if (!c->prof) return nullptr;
  if (!c->prof_only.empty() && (!name || c->prof_only != name)) return nullptr;
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

// Host staging of the fixed contexts: plain static arrays (pageable), one set
// per device, so a fixed context never allocates.
constexpr size_t kFixedPinned = 4u << 20;
constexpr size_t kFixedPinTab = 1u << 20;
static uint8_t g_fixed_pinned[kFixedDevices][kFixedPinned];
static uint8_t g_fixed_pin_tab[kFixedDevices][kFixedPinTab];
static uint8_t g_fixed_pin_pre[kFixedDevices][kPrefixBytes];
static hpez_ctx g_fixed_ctx[kFixedDevices];

int decompress_fixed(int device, void* ws, size_t ws_bytes, const void* d_in, uint64_t in_size,
                     void* d_out, uint64_t out_cap, hipStream_t stream)
{
  if (device < 0 || device >= kFixedDevices || !ws) return HPEZ_EINVAL;
  hpez_ctx* c = &g_fixed_ctx[device];
  c->device = device;
  c->fixed = true;
  c->ws = ws;
  c->ws_bytes = ws_bytes;
  c->pinned = g_fixed_pinned[device];
  c->pinned_bytes = kFixedPinned;
  c->pin_tab = g_fixed_pin_tab[device];
  c->pin_tab_bytes = kFixedPinTab;
  c->pin_pre = g_fixed_pin_pre[device];
  c->pin_pre_bytes = kPrefixBytes;
  return hpez_decompress(c, d_in, in_size, d_out, out_cap, stream);
}

}  // namespace hpez

// ---------------------------------------------------------------------------
// Decompression plans: the device work of one decompression call recorded as
// a HIP graph on a private context, replayed without host work.

struct hpez_plan {
  // private contexts (workspace and staging of the replays): one for the
  // float32 streams, one for the others (float64 arithmetic).  A call's two
  // dtype groups reuse one context's host staging one after the other, which
  // a graph's copy nodes, reading host memory when replayed, cannot share.
  hpez_ctx* pc[2] = {nullptr, nullptr};
  hipStream_t cs = nullptr;  // the stream the graph is recorded on
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int n = 0;
  std::vector<hpez_ctx::Check> checks;  // idx: the stream's index in the plan
  uint8_t* h_res = nullptr;             // pinned: status words and counts read back
  hipEvent_t done = nullptr;            // recorded after every replay (destroy waits on it)
};

namespace {

void plan_free(hpez_plan* p)
{
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cs) (void)hipStreamDestroy(p->cs);
  if (p->h_res) (void)hipHostFree(p->h_res);
  if (p->done) (void)hipEventDestroy(p->done);
  for (hpez_ctx* c : p->pc)
    if (c) hpez_ctx_destroy(c);
  delete p;
}

// true if the graph holds a memset node: the recorded work clears memory only
// by copies and kernels, so such a node means an unexpected call was recorded
bool graph_has_memset(hipGraph_t g)
{
  size_t nn = 0;
  if (hipGraphGetNodes(g, nullptr, &nn) != hipSuccess) return true;
  std::vector<hipGraphNode_t> nodes(nn);
  if (nn && hipGraphGetNodes(g, nodes.data(), &nn) != hipSuccess) return true;
  for (hipGraphNode_t nd : nodes) {
    hipGraphNodeType t;
    if (hipGraphNodeGetType(nd, &t) != hipSuccess || t == hipGraphNodeTypeMemset) return true;
  }
  return false;
}

int plan_device(const hpez_plan* p) { return p->pc[0] ? p->pc[0]->device : p->pc[1]->device; }

// the streams of one dtype group, as hpez_decompress_batch arguments
struct PlanGroup {
  std::vector<int> idx;
  std::vector<const void*> in;
  std::vector<uint64_t> size, cap;
  std::vector<void*> out;
  std::vector<int> rcs;
  int call(hpez_ctx* c, hipStream_t st)
  {
    return hpez_decompress_batch(c, (int)idx.size(), in.data(), size.data(), out.data(), cap.data(),
                                 rcs.data(), st);
  }
};

}  // namespace

extern "C" {

int hpez_decompress_plan(hpez_ctx* ctx, int n, const void* const* d_in, const uint64_t* in_size,
                         void* const* d_out, const uint64_t* out_cap, int* rcs,
                         hipStream_t stream, hpez_plan** out_plan)
{
  if (!out_plan) return HPEZ_EINVAL;
  *out_plan = nullptr;
  if (!ctx || n < 1 || !d_in || !in_size || !d_out || !out_cap || !rcs) return HPEZ_EINVAL;
  for (int i = 0; i < n; i++)
    if (!d_in[i] || !d_out[i]) return HPEZ_EINVAL;
  DevScope ds(ctx->device);
  // headers: the dtype group of every stream
  std::vector<uint8_t> hdr((size_t)n * kHdrBytes, 0);
  for (int i = 0; i < n; i++) {
    rcs[i] = in_size[i] < (uint64_t)kHdrBytes ? HPEZ_ECORRUPT : HPEZ_OK;
    if (!rcs[i])
      HIPCK(hipMemcpyAsync(hdr.data() + (size_t)i * kHdrBytes, d_in[i], kHdrBytes,
                           hipMemcpyDeviceToHost, stream));
  }
  HIPCK(hipStreamSynchronize(stream));
  PlanGroup grp[2];
  for (int i = 0; i < n; i++) {
    hpez_field_desc dd;
    hpez_config cc;
    Layout L;
    if (!rcs[i]) rcs[i] = read_header(hdr.data() + (size_t)i * kHdrBytes, in_size[i], &dd, &cc, &L);
    if (rcs[i]) return rcs[i];
    PlanGroup& G = grp[dd.dtype == HPEZ_F32 ? 0 : 1];
    G.idx.push_back(i);
    G.in.push_back(d_in[i]);
    G.size.push_back(in_size[i]);
    G.out.push_back(d_out[i]);
    G.cap.push_back(out_cap[i]);
    G.rcs.push_back(HPEZ_OK);
  }
  hpez_plan* p = new (std::nothrow) hpez_plan;
  if (!p) return HPEZ_ENOMEM;
  p->n = n;
  // the eager calls: check every stream, fill the outputs and size each
  // group's workspace and staging
  int rc = HPEZ_OK;
  for (int g = 0; g < 2 && !rc; g++) {
    PlanGroup& G = grp[g];
    if (G.idx.empty()) continue;
    rc = hpez_ctx_create(&p->pc[g], ctx->device);
    if (rc) break;
    p->pc[g]->tiles = ctx->tiles;
    rc = G.call(p->pc[g], stream);
    for (size_t k = 0; k < G.idx.size(); k++) rcs[G.idx[k]] = G.rcs[k];
  }
  if (!rc && hipStreamCreateWithFlags(&p->cs, hipStreamNonBlocking) != hipSuccess) rc = HPEZ_EDEVICE;
  if (rc) {
    plan_free(p);
    return rc;
  }
  // the recording: same jobs, same buffers; no growth (fixed), no block-phase
  // second stream; per-field work of several streams forks onto the pool
  // streams the eager call made, which the recording joins as branches
  if (hipStreamBeginCapture(p->cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    plan_free(p);
    return HPEZ_EDEVICE;
  }
  for (int g = 0; g < 2 && !rc; g++) {
    if (!p->pc[g]) continue;
    p->pc[g]->capture = true;
    p->pc[g]->fixed = true;
    rc = grp[g].call(p->pc[g], p->cs);
    p->pc[g]->capture = false;
  }
  hipGraph_t gr = nullptr;
  const hipError_t e = hipStreamEndCapture(p->cs, &gr);
  p->graph = gr;
  if (rc || e != hipSuccess || !gr || graph_has_memset(gr) ||
      hipGraphInstantiateWithFlags(&p->exec, gr, 0) != hipSuccess) {
    plan_free(p);
    return rc ? rc : HPEZ_EDEVICE;
  }
  for (int g = 0; g < 2; g++) {
    if (!p->pc[g]) continue;
    for (hpez_ctx::Check c : p->pc[g]->checks) {
      c.idx = grp[g].idx[c.idx];
      p->checks.push_back(c);
    }
  }
  if (hipHostMalloc((void**)&p->h_res, p->checks.size() * 16 + 16, hipHostMallocDefault) !=
      hipSuccess) {
    p->h_res = nullptr;
    plan_free(p);
    return HPEZ_ENOMEM;
  }
  if (hipEventCreateWithFlags(&p->done, hipEventDisableTiming) != hipSuccess) {
    p->done = nullptr;
    plan_free(p);
    return HPEZ_EDEVICE;
  }
  *out_plan = p;
  return HPEZ_OK;
}

int hpez_plan_launch(hpez_plan* plan, hipStream_t stream)
{
  if (!plan || !plan->exec) return HPEZ_EINVAL;
  DevScope ds(plan_device(plan));
  if (hipGraphLaunch(plan->exec, stream) != hipSuccess ||
      hipEventRecord(plan->done, stream) != hipSuccess)
    return HPEZ_EDEVICE;
  return HPEZ_OK;
}

int hpez_plan_status(hpez_plan* plan, hipStream_t stream, int* rcs)
{
  if (!plan || !rcs) return HPEZ_EINVAL;
  DevScope ds(plan_device(plan));
  const size_t nc = plan->checks.size();
  uint64_t* tot = reinterpret_cast<uint64_t*>(plan->h_res);
  int* status = reinterpret_cast<int*>(plan->h_res + nc * 8);
  for (size_t k = 0; k < nc; k++) {
    const hpez_ctx::Check& c = plan->checks[k];
    HIPCK(hipMemcpyAsync(&status[k], c.status, sizeof(int), hipMemcpyDeviceToHost, stream));
    HIPCK(hipMemcpyAsync(&tot[k], c.tot, 8, hipMemcpyDeviceToHost, stream));
  }
  HIPCK(hipStreamSynchronize(stream));
  for (int i = 0; i < plan->n; i++) rcs[i] = HPEZ_OK;
  for (size_t k = 0; k < nc; k++) {
    const hpez_ctx::Check& c = plan->checks[k];
    if (status[k] || tot[k] != c.want) rcs[c.idx] = HPEZ_ECORRUPT;
  }
  for (int i = 0; i < plan->n; i++)
    if (rcs[i]) return rcs[i];
  return HPEZ_OK;
}

void hpez_plan_destroy(hpez_plan* plan)
{
  if (!plan) return;
  DevScope ds(plan_device(plan));
  // the last replay launched (on whatever stream) ends before the plan's
  // memory is released
  if (plan->done) (void)hipEventSynchronize(plan->done);
  plan_free(plan);
}

}  // extern "C"
