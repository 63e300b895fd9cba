// tune.cpp -- host orchestration of the auto-tuner (Sec. 6) of the MI355X
// HPEZ library.  The heavy parts (sampling statistics, the closed-loop trial
// compressions of every candidate on every sampled region, the Lorenzo trial)
// run in the kernels of k_tune.hip; the host makes the decisions from their
// integer scores and histograms:
//   Sec. 6.1  sigma^2 per kind and dimension -> the Eq. (12) weights 1/sigma^2
//             and the least smooth dimension (the freeze candidate);
//   Sec. 6.2  per level, the candidate with the lowest summed error score on
//             the (B+1)^D boxes of every k-th block, k = round(1 / rate);
//   Sec. 6.3  the same with the freeze candidate frozen; freeze iff the
//             estimated bits per point (entropy of the tuned trial's codes plus
//             the anchors' verbatim bits) is lower;
//   Sec. 6.5  Lorenzo iff coef * (entropy of its trial codes) is lower still;
//   Sec. 6.6  per block, the candidate with the lowest total score on the
//             block's centred sub-block of side round(B * rate^(1/D)).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "hpez_host.h"
#include "tune_dev.h"

using namespace hpez;

namespace {

constexpr int kNCand = 11;

#define TCK(x)                                  \
  do {                                          \
    if ((x) != hipSuccess) return HPEZ_EDEVICE; \
  } while (0)

// The eleven interpolation candidates: {linear, not-a-knot, natural} x
// {1D natural order, 1D reversed order, multi-dimensional}, then not-a-knot and
// natural with same-level cubic in natural order.
void candidate_list(int ndims, hpez_interp* c)
{
  for (int i = 0; i < kNCand; i++) {
    std::memset(&c[i], 0, sizeof c[i]);
    const int kind = i < 9 ? i / 3 : (i == 9 ? 1 : 2);
    const int par = i < 9 ? i % 3 : 0;
    c[i].kind = (uint8_t)kind;
    c[i].md = par == 2 ? 1 : 0;
    c[i].same_level = i >= 9 ? 1 : 0;
    for (int j = 0; j < 4; j++) c[i].order[j] = (uint8_t)j;
    if (par == 1)
      for (int j = 0; j < ndims; j++) c[i].order[j] = (uint8_t)(ndims - 1 - j);
  }
}

// zeroth-order entropy in bits per symbol, summed in ascending symbol order
double entropy_bits(const uint32_t* h, uint32_t nsym)
{
  uint64_t n = 0;
  for (uint32_t k = 0; k < nsym; k++) n += h[k];
  if (n == 0) return 0.0;
  double acc = 0.0;
  for (uint32_t k = 0; k < nsym; k++)
    if (h[k]) acc += (double)h[k] * std::log2((double)n / (double)h[k]);
  return acc / (double)n;
}

// the same estimate from the nonzero bins as (bin, count) pairs in any order:
// sorted by bin, the sums run over the same terms in the same order
double entropy_bits_pairs(const uint32_t* pairs, uint32_t n)
{
  // the sum runs over the bins in increasing order; the bins are distinct and
  // below 2^16 (codes are 16-bit), so two 8-bit radix passes sort the pairs
  std::vector<uint32_t> a(pairs, pairs + 2 * (size_t)n), b(2 * (size_t)n);
  bool small = true;
  for (uint32_t i = 0; i < n; i++) small = small && a[2 * i] < 65536u;
  if (small) {
    for (int pass = 0; pass < 2; pass++) {
      const int sh = 8 * pass;
      uint32_t cnt[257] = {0};
      for (uint32_t i = 0; i < n; i++) cnt[((a[2 * i] >> sh) & 255u) + 1]++;
      for (int k = 0; k < 256; k++) cnt[k + 1] += cnt[k];
      for (uint32_t i = 0; i < n; i++) {
        const uint32_t d = cnt[(a[2 * i] >> sh) & 255u]++;
        b[2 * d] = a[2 * i];
        b[2 * d + 1] = a[2 * i + 1];
      }
      a.swap(b);
    }
  } else {
    std::vector<std::pair<uint32_t, uint32_t>> v(n);
    for (uint32_t i = 0; i < n; i++) v[i] = {a[2 * i], a[2 * i + 1]};
    std::sort(v.begin(), v.end());
    for (uint32_t i = 0; i < n; i++) {
      a[2 * i] = v[i].first;
      a[2 * i + 1] = v[i].second;
    }
  }
  uint64_t tot = 0;
  for (uint32_t i = 0; i < n; i++) tot += a[2 * i + 1];
  if (tot == 0) return 0.0;
  // c log2(tot / c) per bin, summed in bin order; the term of a small count is
  // computed once per count (the same expression, so the same bits): most bins
  // of a trial histogram hold small counts that repeat
  constexpr uint32_t kSmall = 4096;
  static thread_local double term[kSmall];
  static thread_local uint64_t term_tot[kSmall];
  double acc = 0.0;
  for (uint32_t i = 0; i < n; i++) {
    const uint32_t ci = a[2 * i + 1];
    const double c = (double)ci;
    if (ci < kSmall) {
      if (term_tot[ci] != tot + 1) {
        term[ci] = c * std::log2((double)tot / c);
        term_tot[ci] = tot + 1;  // + 1: a zeroed entry never matches
      }
      acc += term[ci];
    } else {
      acc += c * std::log2((double)tot / c);
    }
  }
  return acc / (double)tot;
}

int64_t anchor_count(const hpez_field_desc* d, int frozen, int64_t A)
{
  int64_t c = 1;
  for (int i = 0; i < d->ndims; i++) {
    const int64_t n = (int64_t)d->dims[i];
    c *= (n > 1 && i != frozen) ? (n - 1) / A + 1 : n;
  }
  return c;
}

void unravel(int64_t bi, const int64_t* nb, int64_t* b)
{
  for (int d = 3; d >= 0; d--) {
    b[d] = bi % nb[d];
    bi /= nb[d];
  }
}

// (B+1)^D boxes at the origins of every k-th block
std::vector<TrialBox> global_boxes(const Geom& g, int64_t B, double rate, uint64_t* cap)
{
  int64_t nb[4], nbt = 1;
  for (int d = 0; d < 4; d++) {
    nb[d] = (g.n[d] + B - 1) / B;
    nbt *= nb[d];
  }
  int64_t k = (int64_t)std::floor(1.0 / rate + 0.5);
  if (k < 1) k = 1;
  int64_t first = k / 2;
  if (first >= nbt) first = nbt / 2;
  std::vector<TrialBox> v;
  *cap = 0;
  for (int64_t bi = first; bi < nbt; bi += k) {
    int64_t b[4];
    unravel(bi, nb, b);
    TrialBox t;
    uint64_t pts = 1;
    for (int d = 0; d < 4; d++) {
      t.o[d] = b[d] * B;
      t.m[d] = g.n[d] - t.o[d] < B + 1 ? g.n[d] - t.o[d] : B + 1;
      pts *= (uint64_t)t.m[d];
    }
    *cap = std::max(*cap, pts);
    v.push_back(t);
  }
  return v;
}

void fill_levels(TrialArgs& a, double e, const hpez_config* Q, int dtype)
{
  for (int l = 1; l <= 16; l++) {
    const double el = level_eb(e, Q->alpha, Q->beta, l);
    a.el[l] = el;
    a.inv2e[l] = 1.0 / (2.0 * el);
    a.twoe[l] = twoe_of(el, dtype);
  }
  a.el[0] = a.inv2e[0] = a.twoe[0] = 0.0;
  double wq[3 * 16 * 4];
  md_table(Q, wq);
  for (int k = 0; k < 3; k++)
    for (int odd = 0; odd < 8; odd++)
      for (int d = 0; d < 4; d++) a.wmd[(k * 8 + odd) * 4 + d] = wq[(k * 16 + odd) * 4 + d];
}

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// Longest side of the block-wise sub-blocks (Sec. 6.6) for D active dims.
int64_t sub_side(int64_t B, double rate, int D)
{
  int64_t side = (int64_t)std::floor((double)B * std::pow(rate, 1.0 / (double)D) + 0.5);
  return std::min<int64_t>(std::max<int64_t>(side, 3), B);
}

// Global scratch for regions too large for LDS (the non-box trial kernels).
size_t trial_scratch(const Geom& g, const hpez_tune_opts* o, size_t s, size_t n_global,
                     uint64_t gcap, int64_t nbt)
{
  size_t scratch = gcap * s > kTrialLdsBytes ? n_global * kNCand * gcap * s : 0;
  if (o->block_wise) {
    // largest sub-block: fewest active dims (one frozen) gives the longest side
    int big_dims = 0;
    for (int k = 0; k < 4; k++) big_dims += g.n[k] > 1;
    const int Dmin = n_active(g) > 1 ? n_active(g) - 1 : 1;
    const int64_t side = sub_side((int64_t)1 << o->block_log2, o->sub_rate, Dmin);
    uint64_t bcap_pts = 1;
    for (int k = 0; k < big_dims; k++) bcap_pts *= (uint64_t)side;
    if (bcap_pts * s > kTrialLdsBytes)
      scratch = std::max(scratch, (size_t)nbt * kNCand * bcap_pts * s);
  }
  return scratch;
}

// ---------------------------------------------------------------------------
// Tuning of one field as a job in phases.  The plain call runs one job, the
// batch call many, with one stream synchronization per phase for all of them
// and the trials of every job in fused launches:
//   1. value range;  2. Sec. 6.1 statistics;
//   3. Sec. 6.2 / 6.3 candidate trials, unfrozen and frozen, and the Sec. 6.5
//      Lorenzo trial;  4. the tuned trials' code histograms;
//   5. Sec. 6.6 block-wise trials;  6. decisions.
// Each job takes the same steps either way, so its decisions are the same.
template <typename T>
struct TJob {
  const hpez_field_desc* d = nullptr;
  const T* X = nullptr;
  const hpez_tune_opts* o = nullptr;
  hpez_config* cfg = nullptr;
  uint8_t* h_bcfg = nullptr;
  uint64_t bcap = 0;
  int rc = HPEZ_OK;
  bool done = false;  // finished early (constant field) or failed
  hpez_config Q;
  Geom g;
  int64_t B = 0, nbt = 0;
  uint64_t N = 0;
  uint32_t nsym = 0;
  double e = 0;
  hpez_interp cand[kNCand];
  std::vector<TrialBox> gb;  // global regions
  uint64_t gcap = 0;
  size_t scratch_bytes = 0;
  int nvar = 1;  // global trial variants: unfrozen, then frozen at fcand
  int fcand = -1;
  bool stats = false;
  int64_t count = 0;
  TrialArgs ga[2];
  hpez_interp lv[2][16];
  double H[2] = {0, 0};
  int frozen = -1;
  bool lorenzo = false, lorenzo_trial = false;
  bool blocks = false;
  bool spec = false;  // block trials already queued on the second stream
  // the block trials' boxes, built and uploaded for this freeze decision
  // (bb_frozen) ahead of the trials: box side, anchor level and largest box
  bool bb_ready = false;
  int bb_frozen = -2;
  hipStream_t bb_stream = nullptr;  // the stream their upload is ordered on
  int64_t bb_side = 0;
  int bb_al = 0;
  uint64_t bb_cap = 0;
  double HL = 0.0;     // entropy of the Lorenzo trial's codes
  TrialArgs ba;
  // Sec. 6.4: the (alpha, beta) trials (when tune_ab)
  bool ab = false;      // the trials run for this job
  int nab = 0;          // grid pairs with workspace (kNAB when tune_ab, else 0)
  unsigned long long* absq = nullptr;   // per pair: the distortion
  uint32_t* abhist = nullptr;           // per pair: the codes' histogram (nsym bins)
  uint32_t* abnz = nullptr;             // per pair: its nonzero (bin, count) pairs
  uint32_t* abnzn = nullptr;            // per pair: the pair count
  unsigned long long* h_absq = nullptr;
  uint32_t* h_abnz = nullptr;
  uint32_t* h_abnzn = nullptr;
  uint32_t* h_abhist = nullptr;         // one histogram, read when the pairs overflow
  double h_wq[3 * 16 * 4];
  // device
  TrialBox* d_gb = nullptr;
  TrialBox* d_bb = nullptr;
  void* scratch = nullptr;
  unsigned long long* score[2] = {nullptr, nullptr};
  unsigned long long* bscore = nullptr;
  unsigned long long* dummy = nullptr;
  uint32_t* hist[3] = {nullptr, nullptr, nullptr};
  uint32_t* nz[3] = {nullptr, nullptr, nullptr};  // nonzero (bin, count) pairs per histogram
  int* flag = nullptr;  // [0] non-finite input, [4 + v] pair count of histogram v
  int* lflag = nullptr;
  double* wq = nullptr;
  double* part = nullptr;
  double* mm = nullptr;
  unsigned long long* sums = nullptr;
  // pinned host staging
  uint32_t* h_hist[3] = {nullptr, nullptr, nullptr};
  uint32_t* h_nz[3] = {nullptr, nullptr, nullptr};
  uint32_t* h_nzn = nullptr;  // the three pair counts
  unsigned long long* h_score[2] = {nullptr, nullptr};
  unsigned long long* h_bscore = nullptr;
  double* h_mm = nullptr;
  int* h_bad = nullptr;
  int* h_lflag = nullptr;
  unsigned long long* h_sums = nullptr;
  double* h_wqp = nullptr;    // staging of h_wq
  TrialBox* h_gbp = nullptr;  // staging of gb
};

// The (alpha, beta) grid of Sec. 6.4 (Eq. 15): (1, 1) first, then alpha-major
// over {1.25, 1.5, 1.75, 2} x {1.5, 2, 3, 4}.
constexpr int kNAB = 17;
void ab_pair(int c, double* alpha, double* beta)
{
  static const double av[4] = {1.25, 1.5, 1.75, 2.0}, bv[4] = {1.5, 2.0, 3.0, 4.0};
  if (c == 0) {
    *alpha = *beta = 1.0;
    return;
  }
  *alpha = av[(c - 1) / 4];
  *beta = bv[(c - 1) % 4];
}

// validation and sizes; rc set for a bad request
template <typename T>
void t_init(TJob<T>& J)
{
  const hpez_field_desc* d = J.d;
  const hpez_tune_opts* o = J.o;
  hpez_config& Q = J.Q;
  J.N = points_of(d);
  std::memset(&Q, 0, sizeof Q);
  Q.radius = J.cfg->radius;
  Q.chunk = J.cfg->chunk;
  Q.alpha = J.cfg->alpha;
  Q.beta = J.cfg->beta;
  Q.frozen_dim = -1;
  for (int k = 0; k < 3; k++)
    for (int j = 0; j < 4; j++) Q.md_w[k][j] = 1.0;
  for (int i = 0; i < 16; i++)
    for (int j = 0; j < 4; j++) {
      Q.level[i].order[j] = (uint8_t)j;
      Q.cand[i].order[j] = (uint8_t)j;
    }
  if (check_cfg(d, &Q, false) || o->block_log2 < 1 || o->block_log2 > 8 ||
      !(o->global_rate > 0) || !(o->sub_rate > 0) || !(o->lorenzo_coef > 0)) {
    J.rc = HPEZ_EINVAL;
    J.done = true;
    return;
  }
  int big = 0;
  for (int i = 0; i < d->ndims; i++) big += d->dims[i] > 1;
  Q.anchor_log2 = o->anchor_log2 ? o->anchor_log2 : (big >= 3 ? 6 : big == 2 ? 7 : 8);
  J.g = make_geom(d, -1);
  J.B = (int64_t)1 << o->block_log2;
  J.nbt = 1;
  for (int k = 0; k < 4; k++) J.nbt *= (J.g.n[k] + J.B - 1) / J.B;
  if (o->block_wise && (!J.h_bcfg || J.bcap < (uint64_t)J.nbt)) {
    J.rc = HPEZ_EINVAL;
    J.done = true;
    return;
  }
  J.nsym = 2 * Q.radius;
  J.nab = o->tune_ab ? kNAB : 0;
  candidate_list(d->ndims, J.cand);
  J.gb = global_boxes(J.g, J.B, o->global_rate, &J.gcap);
  J.scratch_bytes = trial_scratch(J.g, o, sizeof(T), J.gb.size(), J.gcap, J.nbt);
}

template <typename T>
size_t t_dev_bytes(const TJob<T>& J)
{
  if (J.done) return 0;
  const size_t nb = (size_t)J.nbt;
  return al256(J.gb.size() * sizeof(TrialBox)) + al256(nb * sizeof(TrialBox)) +
         al256(J.scratch_bytes) + 2 * al256(kNCand * 16 * 8) + al256(nb * kNCand * 8) +
         al256(16 * 8) + 3 * al256(J.nsym * 4) + 3 * al256(kNzCap * 8) + 2 * al256(64) +
         al256(3 * 16 * 4 * 8) +
         al256(2 * 1024 * 8) + al256(64) + al256(12 * 8 * kStatSlots) + 256 +
         al256((size_t)J.nab * 8) + al256((size_t)J.nab * J.nsym * 4) +
         al256((size_t)J.nab * 2 * kNzCap * 4) + al256((size_t)J.nab * 4);
}

template <typename T>
size_t t_pin_bytes(const TJob<T>& J)
{
  if (J.done) return 0;
  return 3 * al256(J.nsym * 4) + 3 * al256(kNzCap * 8) + al256(16) + 2 * al256(kNCand * 16 * 8) +
         al256((size_t)J.nbt * kNCand * 8) + al256(64) + al256(12 * 8 * kStatSlots) +
         al256(3 * 16 * 4 * 8) +
         al256(J.gb.size() * sizeof(TrialBox)) + 256 + al256((size_t)J.nab * 8) +
         al256((size_t)J.nab * 2 * kNzCap * 4) + al256((size_t)J.nab * 4) +
         (J.nab ? al256((size_t)J.nsym * 4) : 0);
}

struct Take {
  uint8_t* base;
  size_t off = 0;
  template <typename U>
  U* take(size_t count)
  {
    U* p = reinterpret_cast<U*>(base + off);
    off += al256(count * sizeof(U));
    return p;
  }
};

template <typename T>
void t_take(TJob<T>& J, Take& dw, Take& pw)
{
  if (J.done) return;
  J.d_gb = dw.take<TrialBox>(J.gb.size());
  J.d_bb = dw.take<TrialBox>((size_t)J.nbt);
  J.scratch = dw.take<uint8_t>(J.scratch_bytes);
  J.score[0] = dw.take<unsigned long long>(kNCand * 16);
  J.score[1] = dw.take<unsigned long long>(kNCand * 16);
  J.bscore = dw.take<unsigned long long>((size_t)J.nbt * kNCand);
  J.dummy = dw.take<unsigned long long>(16);
  J.absq = dw.take<unsigned long long>((size_t)J.nab);
  J.abhist = dw.take<uint32_t>((size_t)J.nab * J.nsym);
  J.abnz = dw.take<uint32_t>((size_t)J.nab * 2 * kNzCap);
  J.abnzn = dw.take<uint32_t>((size_t)J.nab);
  for (int v = 0; v < 3; v++) J.hist[v] = dw.take<uint32_t>(J.nsym);
  for (int v = 0; v < 3; v++) J.nz[v] = dw.take<uint32_t>(2 * kNzCap);
  J.flag = dw.take<int>(16);
  J.lflag = dw.take<int>(16);
  J.wq = dw.take<double>(3 * 16 * 4);
  J.part = dw.take<double>(2 * 1024);
  J.mm = dw.take<double>(8);
  J.sums = dw.take<unsigned long long>(12 * kStatSlots);
  for (int v = 0; v < 3; v++) J.h_hist[v] = pw.take<uint32_t>(J.nsym);
  for (int v = 0; v < 3; v++) J.h_nz[v] = pw.take<uint32_t>(2 * kNzCap);
  J.h_nzn = pw.take<uint32_t>(4);
  J.h_score[0] = pw.take<unsigned long long>(kNCand * 16);
  J.h_score[1] = pw.take<unsigned long long>(kNCand * 16);
  J.h_bscore = pw.take<unsigned long long>((size_t)J.nbt * kNCand);
  J.h_mm = pw.take<double>(8);
  J.h_bad = (int*)(J.h_mm + 2);
  J.h_lflag = (int*)(J.h_mm + 3);
  J.h_sums = pw.take<unsigned long long>(12 * kStatSlots);
  J.h_wqp = pw.take<double>(3 * 16 * 4);
  J.h_gbp = pw.take<TrialBox>(J.gb.size());
  J.h_absq = pw.take<unsigned long long>((size_t)J.nab);
  J.h_abnz = pw.take<uint32_t>((size_t)J.nab * 2 * kNzCap);
  J.h_abnzn = pw.take<uint32_t>((size_t)J.nab);
  if (J.nab) J.h_abhist = pw.take<uint32_t>(J.nsym);
}

// phase 1: value range and the non-finite check
template <typename T>
int t_minmax(TJob<T>& J, hipStream_t st)
{
  if (J.done) return HPEZ_OK;
  // every accumulator and flag of the call (trial scores, histograms, pair
  // counts, flags, statistics sums) lies between score[0] and the end of sums
  // in the workspace: one clear for all of them
  uint8_t* z0 = reinterpret_cast<uint8_t*>(J.score[0]);
  uint8_t* z1 = reinterpret_cast<uint8_t*>(J.sums + 12 * kStatSlots);
  TCK(hipMemsetAsync(z0, 0, (size_t)(z1 - z0), st));
  TCK(launch_minmax<T>(J.X, J.N, J.part, J.flag, 1024, st));
  TCK(launch_minmax_final(J.part, 1024, J.mm, st));
  TCK(hipMemcpyAsync(J.h_mm, J.mm, 16, hipMemcpyDeviceToHost, st));
  TCK(hipMemcpyAsync(J.h_bad, J.flag, 4, hipMemcpyDeviceToHost, st));
  return HPEZ_OK;
}

// phase 2: error bound, constant fields, Sec. 6.1 statistics
template <typename T>
int t_stats(hpez_ctx* ctx, TJob<T>& J, hipStream_t st)
{
  if (J.done) return HPEZ_OK;
  const hpez_field_desc* d = J.d;
  if (*J.h_bad) {
    J.rc = HPEZ_EINVAL;
    J.done = true;
    return HPEZ_OK;
  }
  bool constant = false;
  if (d->eb_mode == HPEZ_REL) {
    const double range = J.h_mm[1] - J.h_mm[0];
    if (range == 0) constant = true;
    J.e = d->eb * range;
  } else {
    J.e = d->eb;
  }
  if (constant) {
    *J.cfg = J.Q;
    J.cfg->n_cand = 0;
    J.cfg->block_cfg = nullptr;
    for (int l = 0; l < 16; l++) J.cfg->level[l] = J.cand[0];
    J.done = true;
    return HPEZ_OK;
  }
  if (!(J.e > 0)) {
    J.rc = HPEZ_EINVAL;
    J.done = true;
    return HPEZ_OK;
  }
  Geom gs = J.g;
  for (int k = 0; k < 4; k++)
    if (gs.act[k] && gs.n[k] < 8) gs.act[k] = 0;
  int any = 0;
  for (int k = 0; k < 4; k++) any |= gs.act[k];
  std::memset(J.h_sums, 0, 12 * 8 * kStatSlots);
  J.count = 0;
  if (!any) return HPEZ_OK;
  Lattice lat;
  lat.total = 1;
  for (int k = 0; k < 4; k++) {
    const int64_t r = gs.act[k] ? 4 : 0, m = gs.act[k] ? 8 : 1;
    const int64_t hi = gs.act[k] ? gs.n[k] - 4 : gs.n[k] - 1;
    lat.first[k] = r;
    lat.step[k] = m;
    lat.cnt[k] = r <= hi ? (uint32_t)((hi - r) / m + 1) : 0;
    lat.total *= lat.cnt[k];
  }
  J.count = (int64_t)lat.total;
  J.stats = true;
  hipEvent_t ev = ctx_span_begin(ctx, st, "tune_stats");
  TCK(launch_stats<T>(J.X, gs, lat, 256.0 / J.e, J.sums, st));
  ctx_span_end(ctx, ev, "tune_stats", lat.total * (1 + 4 * n_active(gs)) * sizeof(T), st);
  TCK(hipMemcpyAsync(J.h_sums, J.sums, 12 * 8 * kStatSlots, hipMemcpyDeviceToHost, st));
  return HPEZ_OK;
}

// Trial launches of a phase: box-eligible entries of all jobs fused (one launch
// per lane count), the others one by one.
template <typename T>
struct TrialBatch {
  hpez_ctx* ctx = nullptr;          // lanes per region size class (hpez_autotune)
  std::vector<TrialJob<T>> grp[3];  // by lanes per work-group: 64, 256, 1024
  struct Single {
    TrialArgs a;
    const TrialBox* boxes;
    uint32_t n_boxes, n_cand;
    const T* X;
    T* scratch;
    const double* wq;
    unsigned long long* score;
    uint32_t* hist;
  };
  std::vector<Single> single;
};

template <typename T>
void t_add(TrialBatch<T>& tb, const TrialArgs& a, const TrialBox* boxes, uint32_t n_boxes,
           uint32_t n_cand, const T* X, T* scratch, const double* wq, unsigned long long* score,
           uint32_t* hist)
{
  if (!n_boxes || !n_cand) return;
  if (trial_box_ok<T>(a, hist != nullptr)) {
    TrialJob<T> j;
    j.a = a;
    j.boxes = boxes;
    j.X = X;
    j.score = score;
    j.hist = hist;
    j.n_boxes = n_boxes;
    j.n_cand = n_cand;
    j.wg_begin = 0;
    int lanes = trial_lanes(a.box_cap);
    if (tb.ctx)
      lanes = (int)ctx_tile(tb.ctx, kTileTrial, sizeof(T) == 4 ? 0 : 1, a.box_cap, (uint32_t)lanes);
    tb.grp[lanes == 64 ? 0 : lanes == 256 ? 1 : 2].push_back(j);
  } else {
    tb.single.push_back({a, boxes, n_boxes, n_cand, X, scratch, wq, score, hist});
  }
}

// stage the tables through pinned memory (one copy) and launch
template <typename T>
int t_launch(hpez_ctx* ctx, TrialBatch<T>& tb, bool hist, uint8_t* d_tab, size_t tab_cap,
             hipStream_t st, uint8_t* h_stage = nullptr)
{
  std::vector<TrialJob<T>>* groups[3] = {&tb.grp[0], &tb.grp[1], &tb.grp[2]};
  const int lanes_of[3] = {64, 256, 1024};
  size_t bytes = 0;
  for (auto* gr : groups) bytes += al256(gr->size() * sizeof(TrialJob<T>)) + al256((gr->size() + 1) * 8);
  if (bytes > tab_cap) return HPEZ_EINVAL;
  if (bytes) {
    int rc;
    uint8_t* h = h_stage ? h_stage : ctx_pin_tab(ctx, bytes, &rc);
    if (!h_stage && rc) return rc;
    size_t off = 0;
    size_t offs[3][2];
    uint64_t tot[3];
    size_t lds[3];
    for (int k = 0; k < 3; k++) {
      auto& gr = *groups[k];
      uint64_t w = 0;
      lds[k] = 0;
      uint64_t* wb = (uint64_t*)(h + off + al256(gr.size() * sizeof(TrialJob<T>)));
      for (size_t i = 0; i < gr.size(); i++) {
        gr[i].wg_begin = w;
        wb[i] = w;
        w += (uint64_t)gr[i].n_boxes * gr[i].n_cand;
        lds[k] = std::max(lds[k], trial_box_lds<T>(gr[i].a, hist));
      }
      wb[gr.size()] = w;
      std::memcpy(h + off, gr.data(), gr.size() * sizeof(TrialJob<T>));
      offs[k][0] = off;
      offs[k][1] = off + al256(gr.size() * sizeof(TrialJob<T>));
      off = offs[k][1] + al256((gr.size() + 1) * 8);
      tot[k] = w;
    }
    TCK(hipMemcpyAsync(d_tab, h, bytes, hipMemcpyHostToDevice, st));
    for (int k = 0; k < 3; k++)
      TCK(launch_trial_jobs<T>((const TrialJob<T>*)(d_tab + offs[k][0]),
                               (const uint64_t*)(d_tab + offs[k][1]), (int)groups[k]->size(),
                               tot[k], lds[k], hist, lanes_of[k], st));
  }
  for (auto& s : tb.single)
    TCK(launch_trials<T>(s.a, s.boxes, s.n_boxes, s.n_cand, s.X, s.scratch, s.wq, s.score, s.hist,
                         st));
  return HPEZ_OK;
}

// phase 3: weights (Eq. 12), the freeze candidate, global trials of both
// variants (Sec. 6.2 / 6.3) and the Lorenzo trial (Sec. 6.5)
template <typename T>
int t_global(TJob<T>& J, TrialBatch<T>& tb, hipStream_t st)
{
  if (J.done) return HPEZ_OK;
  hpez_config& Q = J.Q;
  const hpez_tune_opts* o = J.o;
  double sigma2[3][4];
  for (int k = 0; k < 3; k++)
    for (int j = 0; j < 4; j++) {
      unsigned long long sum = 0;
      for (int c = 0; c < kStatSlots; c++) sum += J.h_sums[c * 12 + k * 4 + j];
      const double s2 = J.count > 0 ? (double)sum / (double)J.count : 1.0;
      sigma2[k][j] = s2;
      Q.md_w[k][j] = 1.0 / (s2 > 1.0 ? s2 : 1.0);
    }
  J.fcand = -1;
  if (J.count > 0 && n_active(J.g) >= 2) {
    for (int k = 0; k < 4; k++)
      if (J.g.act[k] && J.g.n[k] >= 8 && (J.fcand < 0 || sigma2[0][k] > sigma2[0][J.fcand]))
        J.fcand = k;
  }
  md_table(&Q, J.h_wq);
  std::memcpy(J.h_wqp, J.h_wq, sizeof J.h_wq);
  std::memcpy(J.h_gbp, J.gb.data(), J.gb.size() * sizeof(TrialBox));
  TCK(hipMemcpyAsync(J.wq, J.h_wqp, sizeof J.h_wq, hipMemcpyHostToDevice, st));
  TCK(hipMemcpyAsync(J.d_gb, J.h_gbp, J.gb.size() * sizeof(TrialBox), hipMemcpyHostToDevice, st));
  J.nvar = (o->allow_freeze && J.fcand >= 0) ? 2 : 1;
  const uint32_t nbx = (uint32_t)J.gb.size();
  for (int v = 0; v < J.nvar; v++) {
    TrialArgs& a = J.ga[v];
    std::memset(&a, 0, sizeof a);
    a.fg = J.g;
    a.frozen = v == 0 ? -1 : J.fcand;
    a.L = o->block_log2;
    a.R = Q.radius;
    a.box_cap = J.gcap;
    a.max_ext = (int32_t)std::min<int64_t>(J.B + 1, INT32_MAX);
    a.score_mul = 4096.0 / J.e;
    fill_levels(a, J.e, &Q, J.d->dtype);
    for (int i = 0; i < kNCand; i++) a.cand[i] = J.cand[i];
    t_add<T>(tb, a, J.d_gb, nbx, kNCand, J.X, (T*)J.scratch, J.wq, J.score[v], nullptr);
  }
  J.lorenzo_trial = o->allow_lorenzo != 0 && !dtype_int(J.d->dtype);  // integers: interpolation
  return HPEZ_OK;
}

template <typename T>
int t_lorenzo(TJob<T>& J, hipStream_t st)
{
  if (J.done || !J.lorenzo_trial) return HPEZ_OK;
  TCK(launch_lorenzo_trial<T>(J.g, J.d_gb, (uint32_t)J.gb.size(), (uint32_t)J.gcap, J.X,
                              1.0 / (2.0 * J.e), J.Q.radius, trial_hist_lo(J.Q.radius), J.hist[2],
                              J.lflag, st));
  return HPEZ_OK;
}

// histogram v to the host as its nonzero (bin, count) pairs
template <typename T>
hipError_t t_nonzero_copy(TJob<T>& J, int v, hipStream_t st)
{
  uint32_t* cnt = reinterpret_cast<uint32_t*>(J.flag) + 4 + v;
  hipError_t e = launch_hist_nonzero(J.hist[v], J.nsym, cnt, J.nz[v], kNzCap, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(J.h_nz[v], J.nz[v], (size_t)kNzCap * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(J.h_nzn + v, cnt, 4, hipMemcpyDeviceToHost, st);
  return e;
}

// entropy of histogram v from its pairs (after the phase's synchronization);
// the whole histogram is read when the pairs overflowed
template <typename T>
int t_entropy(TJob<T>& J, int v, hipStream_t st, double* H)
{
  if (J.h_nzn[v] <= kNzCap) {
    *H = entropy_bits_pairs(J.h_nz[v], J.h_nzn[v]);
    return HPEZ_OK;
  }
  TCK(hipMemcpyAsync(J.h_hist[v], J.hist[v], sizeof(uint32_t) * J.nsym, hipMemcpyDeviceToHost, st));
  TCK(hipStreamSynchronize(st));
  *H = entropy_bits(J.h_hist[v], J.nsym);
  return HPEZ_OK;
}

template <typename T>
int t_global_copy(TJob<T>& J, hipStream_t st)
{
  if (J.done) return HPEZ_OK;
  for (int v = 0; v < J.nvar; v++)
    TCK(hipMemcpyAsync(J.h_score[v], J.score[v], sizeof(unsigned long long) * kNCand * 16,
                       hipMemcpyDeviceToHost, st));
  if (J.lorenzo_trial) {
    TCK(t_nonzero_copy(J, 2, st));
    TCK(hipMemcpyAsync(J.h_lflag, J.lflag, sizeof(int), hipMemcpyDeviceToHost, st));
  }
  return HPEZ_OK;
}

// phase 4: per level the best candidate, then the tuned trials' histograms
template <typename T>
int t_hist(TJob<T>& J, TrialBatch<T>& tb, hipStream_t st)
{
  if (J.done) return HPEZ_OK;
  const int Lb = J.o->block_log2;
  const int L = J.Q.anchor_log2;
  for (int v = 0; v < J.nvar; v++) {
    int best[17];
    for (int l = 1; l <= Lb; l++) {
      best[l] = 0;
      for (int ci = 1; ci < kNCand; ci++)
        if (J.h_score[v][ci * 16 + l - 1] < J.h_score[v][best[l] * 16 + l - 1]) best[l] = ci;
    }
    TrialArgs a = J.ga[v];
    a.tuned = 1;
    a.hist_lo = trial_hist_lo(J.Q.radius);
    for (int l = 1; l <= Lb; l++) a.level[l - 1] = J.cand[best[l]];
    for (int l = 1; l <= 16; l++) {
      const int lb = l <= Lb ? l : Lb;
      J.lv[v][l - 1] = l <= L ? J.cand[best[lb]] : J.cand[0];
    }
    t_add<T>(tb, a, J.d_gb, (uint32_t)J.gb.size(), 1, J.X, (T*)J.scratch, J.wq, J.dummy, J.hist[v]);
  }
  return HPEZ_OK;
}

template <typename T>
int t_hist_copy(TJob<T>& J, hipStream_t st)
{
  if (J.done) return HPEZ_OK;
  for (int v = 0; v < J.nvar; v++) TCK(t_nonzero_copy(J, v, st));
  return HPEZ_OK;
}

// phase 5: freeze and Lorenzo decisions, then the block-wise trials (Sec. 6.6)
// the block-wise trials of variant `frozen`: boxes staged in the pinned
// block-score area (read only after the phase's synchronization) and queued for
// upload on st, arguments in J.ba.  Nothing is queued when `need_tables` is set
// and the trials would not run from the job tables (they would use the shared
// scratch area); *ok tells which.
// The block-wise trials' boxes (Sec. 6.6): the centred sub-block of every
// block, staged in h_bscore (free until the trials' scores come back) and
// uploaded on st.  They depend on the freeze decision only (through the number
// of active dims), so the batch builds them while the (alpha, beta) trials run.
template <typename T>
int t_block_boxes(TJob<T>& J, int frozen, hipStream_t st)
{
  const Geom& g = J.g;
  const Geom gf = make_geom(J.d, frozen);
  const int64_t B = J.B;
  int64_t nb[4];
  for (int k = 0; k < 4; k++) nb[k] = (g.n[k] + B - 1) / B;
  const int nact = n_active(gf);
  const int64_t side = sub_side(B, J.o->sub_rate, nact > 0 ? nact : 1);
  int64_t As = 1;
  int al = 0;
  while (As * 2 <= side - 1) {
    As *= 2;
    al++;
  }
  static_assert(sizeof(unsigned long long) * kNCand >= sizeof(TrialBox), "box staging");
  TrialBox* bx = reinterpret_cast<TrialBox*>(J.h_bscore);
  uint64_t cap = 0;
  // blocks in row-major order: the block index advanced like an odometer
  int64_t b[4] = {0, 0, 0, 0};
  for (int64_t bi = 0; bi < J.nbt; bi++) {
    uint64_t pts = 1;
    for (int k = 0; k < 4; k++) {
      const int64_t ext = g.n[k] - b[k] * B < B ? g.n[k] - b[k] * B : B;
      bx[bi].m[k] = g.n[k] > 1 ? (side < ext ? side : ext) : 1;
      bx[bi].o[k] = b[k] * B + (ext - bx[bi].m[k]) / 2;
      pts *= (uint64_t)bx[bi].m[k];
    }
    cap = std::max(cap, pts);
    for (int k = 3; k >= 0; k--) {
      if (++b[k] < nb[k]) break;
      b[k] = 0;
    }
  }
  TCK(hipMemcpyAsync(J.d_bb, J.h_bscore, (size_t)J.nbt * sizeof(TrialBox), hipMemcpyHostToDevice,
                     st));
  J.bb_ready = true;
  J.bb_frozen = frozen;
  J.bb_stream = st;
  J.bb_side = side;
  J.bb_al = al;
  J.bb_cap = cap;
  return HPEZ_OK;
}

template <typename T>
int t_block_args(TJob<T>& J, int frozen, TrialBatch<T>& tb, hipStream_t st, bool need_tables,
                 bool* ok)
{
  *ok = false;
  if (!(J.bb_ready && J.bb_frozen == frozen && J.bb_stream == st)) {
    const int rc = t_block_boxes(J, frozen, st);
    if (rc) return rc;
  }
  const Geom& g = J.g;
  const int64_t side = J.bb_side;
  const int al = J.bb_al;
  const uint64_t cap = J.bb_cap;
  if ((size_t)J.nbt * kNCand * cap * sizeof(T) > J.scratch_bytes && cap * sizeof(T) > kTrialLdsBytes)
    return need_tables ? HPEZ_OK : HPEZ_ENOMEM;
  TrialArgs& a = J.ba;
  std::memset(&a, 0, sizeof a);
  a.fg = g;
  a.frozen = frozen;
  a.L = al;
  a.R = J.Q.radius;
  a.score_mode = 1;
  a.box_cap = cap;
  a.max_ext = (int32_t)side;
  a.score_mul = 4096.0 / J.e;
  fill_levels(a, J.e, &J.Q, J.d->dtype);
  for (int i = 0; i < kNCand; i++) a.cand[i] = J.cand[i];
  if (need_tables && !trial_box_ok<T>(a, false)) return HPEZ_OK;
  t_add<T>(tb, a, J.d_bb, (uint32_t)J.nbt, kNCand, J.X, (T*)J.scratch, J.wq, J.bscore, nullptr);
  *ok = true;
  return HPEZ_OK;
}

// Block-wise trials queued ahead on the second stream.  With one global
// variant (no freeze candidate) they depend only on the statistics phase: the
// later phases decide only whether their scores are used (not when the Lorenzo
// predictor wins).
template <typename T>
int t_blocks_ahead(TJob<T>& J, TrialBatch<T>& tb, hipStream_t side)
{
  if (J.done || J.nvar != 1 || !J.o->block_wise || !J.nbt || J.nab) return HPEZ_OK;
  bool ok = false;
  const int rc = t_block_args(J, -1, tb, side, true, &ok);
  if (rc) return rc;
  J.spec = ok;
  return HPEZ_OK;
}

// phase 5: the freeze (Sec. 6.3) and Lorenzo (Sec. 6.5) decisions
template <typename T>
int t_decide(TJob<T>& J, hipStream_t st)
{
  if (J.done) return HPEZ_OK;
  const hpez_field_desc* d = J.d;
  const hpez_tune_opts* o = J.o;
  const int64_t A = (int64_t)1 << J.Q.anchor_log2;
  int rc;
  for (int v = 0; v < J.nvar; v++) {
    const int fz = v == 0 ? -1 : J.fcand;
    double Hv;
    if ((rc = t_entropy(J, v, st, &Hv))) return rc;
    J.H[v] = Hv + (double)anchor_count(d, fz, A) * (double)sizeof(T) * 8.0 / (double)points_of(d);
  }
  J.frozen = (J.nvar == 2 && J.H[1] < J.H[0]) ? J.fcand : -1;
  const double Hbest = J.frozen >= 0 ? J.H[1] : J.H[0];
  J.lorenzo = false;
  if (J.lorenzo_trial && *J.h_lflag == 0 && o->lorenzo_coef * J.HL < Hbest) J.lorenzo = true;
  J.blocks = !J.lorenzo && o->block_wise;
  J.ab = !J.lorenzo && J.nab > 0;
  return HPEZ_OK;
}

// phase 6 (tune_ab): the tuned configuration under every (alpha, beta) pair
// of the grid on the global regions (Sec. 6.4, Eq. 15), each pair a trial job
// of its own (its level bounds), its codes' histogram and its distortion
template <typename T>
int t_ab(TJob<T>& J, TrialBatch<T>& tb, hipStream_t st)
{
  if (J.done || !J.ab) return HPEZ_OK;
  const int v = J.frozen >= 0 ? 1 : 0;
  const int Lb = J.o->block_log2;
  for (int c = 0; c < kNAB; c++) {
    TrialArgs a = J.ga[v];
    a.tuned = 1;
    a.score_mode = 2;
    a.inv_e = 1.0 / J.e;
    a.hist_lo = trial_hist_lo(J.Q.radius);
    for (int l = 1; l <= Lb; l++) a.level[l - 1] = J.lv[v][l - 1];
    hpez_config q = J.Q;
    ab_pair(c, &q.alpha, &q.beta);
    fill_levels(a, J.e, &q, J.d->dtype);
    t_add<T>(tb, a, J.d_gb, (uint32_t)J.gb.size(), 1, J.X, (T*)J.scratch, J.wq, J.absq + c,
             J.abhist + (size_t)c * J.nsym);
  }
  return HPEZ_OK;
}

template <typename T>
int t_ab_copy(TJob<T>& J, hipStream_t st)
{
  if (J.done || !J.ab) return HPEZ_OK;
  TCK(launch_hist_nonzero_set(J.abhist, J.nsym, kNAB, J.abnzn, J.abnz, kNzCap, st));
  TCK(hipMemcpyAsync(J.h_abnz, J.abnz, (size_t)kNAB * 2 * kNzCap * 4, hipMemcpyDeviceToHost, st));
  TCK(hipMemcpyAsync(J.h_abnzn, J.abnzn, (size_t)kNAB * 4, hipMemcpyDeviceToHost, st));
  TCK(hipMemcpyAsync(J.h_absq, J.absq, (size_t)kNAB * 8, hipMemcpyDeviceToHost, st));
  return HPEZ_OK;
}

// the pair with the best rate-distortion score: rate = code entropy plus the
// verbatim bits of unpredictable points (code 0) per predicted point, quality
// -10 log10((D + 1) / (n 2^32)) in dB against e, score = quality - 20 log10(2)
// dB per bit (the high-rate slope of a uniform quantizer); ties keep the
// earlier pair
template <typename T>
int t_ab_decide(TJob<T>& J, hipStream_t st)
{
  if (J.done || !J.ab) return HPEZ_OK;
  int best = 0;
  double best_score = 0.0;
  for (int c = 0; c < kNAB; c++) {
    const uint32_t* pairs = J.h_abnz + (size_t)c * 2 * kNzCap;
    const uint32_t np = J.h_abnzn[c];
    uint64_t n = 0, zero = 0;
    double H;
    if (np <= kNzCap) {
      for (uint32_t i = 0; i < np; i++) {
        n += pairs[2 * i + 1];
        if (pairs[2 * i] == 0) zero = pairs[2 * i + 1];
      }
      H = entropy_bits_pairs(pairs, np);
    } else {
      TCK(hipMemcpyAsync(J.h_abhist, J.abhist + (size_t)c * J.nsym, sizeof(uint32_t) * J.nsym,
                         hipMemcpyDeviceToHost, st));
      TCK(hipStreamSynchronize(st));
      for (uint32_t k = 0; k < J.nsym; k++) n += J.h_abhist[k];
      zero = J.h_abhist[0];
      H = entropy_bits(J.h_abhist, J.nsym);
    }
    const double rate = n ? H + (double)zero * (double)sizeof(T) * 8.0 / (double)n : 0.0;
    const double quality =
        n ? -10.0 * std::log10(((double)J.h_absq[c] + 1.0) / ((double)n * 4294967296.0)) : 0.0;
    const double score = quality - 20.0 * std::log10(2.0) * rate;
    if (c == 0 || score > best_score) {
      best = c;
      best_score = score;
    }
  }
  ab_pair(best, &J.Q.alpha, &J.Q.beta);
  return HPEZ_OK;
}

// phase 7: the block-wise trials (Sec. 6.6) with the final level bounds
template <typename T>
int t_blocks(TJob<T>& J, TrialBatch<T>& tb, hipStream_t st)
{
  if (J.done || !J.blocks || J.spec) return HPEZ_OK;
  bool ok = false;
  return t_block_args(J, J.frozen, tb, st, false, &ok);
}

template <typename T>
int t_blocks_copy(TJob<T>& J, hipStream_t st)
{
  if (J.done || !J.blocks || J.spec) return HPEZ_OK;
  TCK(hipMemcpyAsync(J.h_bscore, J.bscore, (size_t)J.nbt * kNCand * sizeof(unsigned long long),
                     hipMemcpyDeviceToHost, st));
  return HPEZ_OK;
}

// phase 6: the configuration
template <typename T>
void t_finish(TJob<T>& J)
{
  if (J.done) return;
  hpez_config out = J.Q;
  out.frozen_dim = (int8_t)(J.lorenzo ? -1 : J.frozen);
  out.predictor = J.lorenzo ? HPEZ_LORENZO : HPEZ_INTERP;
  for (int l = 0; l < 16; l++) out.level[l] = J.lv[J.frozen >= 0 ? 1 : 0][l];
  out.n_cand = 0;
  out.block_cfg = nullptr;
  if (J.blocks) {
    for (int64_t bi = 0; bi < J.nbt; bi++) {
      const unsigned long long* h = J.h_bscore + (size_t)bi * kNCand;
      int besti = 0;
      for (int ci = 1; ci < kNCand; ci++)
        if (h[ci] < h[besti]) besti = ci;
      J.h_bcfg[bi] = (uint8_t)besti;
    }
    out.block_log2 = J.o->block_log2;
    out.n_cand = kNCand;
    for (int i = 0; i < kNCand; i++) out.cand[i] = J.cand[i];
    out.block_cfg = J.h_bcfg;
  }
  *J.cfg = out;
}

template <typename T>
int tune_jobs(hpez_ctx* ctx, std::vector<TJob<T>>& jobs, hipStream_t st)
{
  if (jobs.empty()) return HPEZ_OK;
  size_t dev = 0, pin = 0;
  for (auto& J : jobs) {
    t_init(J);
    dev += t_dev_bytes(J);
    pin += t_pin_bytes(J);
  }
  // trial tables: two global variants per job, or the (alpha, beta) grid, is
  // the most of any phase
  size_t per_job = 2;
  for (auto& J : jobs) per_job = std::max<size_t>(per_job, (size_t)J.nab);
  const size_t tab_cap = al256(per_job * jobs.size() * sizeof(TrialJob<T>)) * 3 +
                         3 * al256((per_job * jobs.size() + 1) * 8) + 512;
  // (a second table, device and pinned staging, for the block trials queued ahead)
  dev += 2 * tab_cap;
  pin += tab_cap;
  int rc;
  uint8_t* base = (uint8_t*)ctx_ws(ctx, dev, &rc);
  if (rc) return rc;
  uint8_t* pbase = ctx_pin(ctx, pin, &rc);
  if (rc) return rc;
  Take dw{base}, pw{pbase};
  uint8_t* d_tab = dw.take<uint8_t>(tab_cap);
  uint8_t* d_tab2 = dw.take<uint8_t>(tab_cap);
  uint8_t* h_tab2 = pw.take<uint8_t>(tab_cap);
  for (auto& J : jobs) t_take(J, dw, pw);
  // whatever way this function returns, the caller's stream waits for the
  // work queued on the second stream
  struct Join {
    hpez_ctx* c;
    hipStream_t st;
    bool on = false;
    ~Join()
    {
      if (on) (void)ctx_join(c, st);
    }
  } join{ctx, st};

  // per-field launches of several fields on the context's stream pool
  const int nj = (int)jobs.size();
  hipStream_t ps[4];
  int np = ctx_fork_pool(ctx, st, nj, ps);
  if (np < 0) return HPEZ_EDEVICE;
  auto js = [&](int i) { return np ? ps[i % np] : st; };
  for (int i = 0; i < nj; i++)
    if ((rc = t_minmax(jobs[i], js(i)))) return rc;
  if (np && (rc = ctx_join_pool(ctx, st, np))) return rc;
  TCK(hipStreamSynchronize(st));
  bool any_stats = false;
  np = ctx_fork_pool(ctx, st, nj, ps);
  if (np < 0) return HPEZ_EDEVICE;
  for (int i = 0; i < nj; i++) {
    if ((rc = t_stats(ctx, jobs[i], js(i)))) return rc;
    any_stats |= jobs[i].stats;
  }
  if (np && (rc = ctx_join_pool(ctx, st, np))) return rc;
  if (any_stats) TCK(hipStreamSynchronize(st));
  {
    TrialBatch<T> tb;
    tb.ctx = ctx;
    for (auto& J : jobs)
      if ((rc = t_global(J, tb, st))) return rc;
    bool ahead = false;
    for (auto& J : jobs) ahead |= !J.done && J.nvar == 1 && J.o->block_wise && J.nbt > 0 && !J.nab;
    hipStream_t side = ahead ? ctx_fork(ctx, st) : nullptr;
    if (side) {
      join.on = true;
      TrialBatch<T> sb;
      sb.ctx = ctx;
      for (auto& J : jobs)
        if ((rc = t_blocks_ahead(J, sb, side))) return rc;
      hipEvent_t evb = ctx_span_begin(ctx, side, "tune_block_trials");
      if ((rc = t_launch(ctx, sb, false, d_tab2, tab_cap, side, h_tab2))) return rc;
      uint64_t bb = 0;
      for (auto& J : jobs)
        if (J.spec) {
          bb += (uint64_t)J.nbt * J.ba.box_cap * sizeof(T);
          TCK(hipMemcpyAsync(J.h_bscore, J.bscore, (size_t)J.nbt * kNCand * sizeof(unsigned long long),
                             hipMemcpyDeviceToHost, side));
        }
      ctx_span_end(ctx, evb, "tune_block_trials", bb, side);
    }
    // the fields' Lorenzo trials on the pool (one stream even for one field),
    // beside the fused trial launch
    bool any_lz = false;
    for (auto& J : jobs) any_lz |= !J.done && J.lorenzo_trial;
    np = any_lz ? ctx_fork_pool(ctx, st, nj > 2 ? nj : 2, ps) : 0;
    if (np < 0) return HPEZ_EDEVICE;
    for (int i = 0; i < nj; i++)
      if ((rc = t_lorenzo(jobs[i], js(i)))) return rc;
    hipEvent_t ev = ctx_span_begin(ctx, st, "tune_trials");
    if ((rc = t_launch(ctx, tb, false, d_tab, tab_cap, st))) return rc;
    uint64_t bytes = 0;
    for (auto& J : jobs)
      if (!J.done) bytes += (uint64_t)J.nvar * J.gb.size() * J.gcap * sizeof(T);
    ctx_span_end(ctx, ev, "tune_trials", bytes, st);
    if (np && (rc = ctx_join_pool(ctx, st, np))) return rc;
    for (auto& J : jobs)
      if ((rc = t_global_copy(J, st))) return rc;
  }
  TCK(hipStreamSynchronize(st));
  {
    TrialBatch<T> tb;
    tb.ctx = ctx;
    for (auto& J : jobs)
      if ((rc = t_hist(J, tb, st))) return rc;
    if ((rc = t_launch(ctx, tb, true, d_tab, tab_cap, st))) return rc;
    for (auto& J : jobs)
      if ((rc = t_hist_copy(J, st))) return rc;
    // the Lorenzo trial's entropy (its pairs arrived with the last phase)
    // while the device runs this one
    for (auto& J : jobs)
      if (!J.done && J.lorenzo_trial && (rc = t_entropy(J, 2, st, &J.HL))) return rc;
  }
  TCK(hipStreamSynchronize(st));
  bool any_ab = false;
  for (auto& J : jobs) {
    if ((rc = t_decide(J, st))) return rc;
    any_ab |= !J.done && J.ab;
  }
  if (any_ab) {
    TrialBatch<T> tb;
    tb.ctx = ctx;
    for (auto& J : jobs)
      if ((rc = t_ab(J, tb, st))) return rc;
    hipEvent_t ev = ctx_span_begin(ctx, st, "tune_ab_trials");
    if ((rc = t_launch(ctx, tb, true, d_tab, tab_cap, st))) return rc;
    uint64_t bytes = 0;
    for (auto& J : jobs)
      if (!J.done && J.ab) bytes += (uint64_t)kNAB * J.gb.size() * J.gcap * sizeof(T);
    ctx_span_end(ctx, ev, "tune_ab_trials", bytes, st);
    for (auto& J : jobs)
      if ((rc = t_ab_copy(J, st))) return rc;
    // the block trials' boxes on the host while the (alpha, beta) trials run
    for (auto& J : jobs)
      if (!J.done && J.blocks && !J.spec && (rc = t_block_boxes(J, J.frozen, st))) return rc;
    TCK(hipStreamSynchronize(st));
    for (auto& J : jobs)
      if ((rc = t_ab_decide(J, st))) return rc;
  }
  {
    TrialBatch<T> tb;
    tb.ctx = ctx;
    for (auto& J : jobs)
      if ((rc = t_blocks(J, tb, st))) return rc;
    hipEvent_t ev = ctx_span_begin(ctx, st, "tune_block_trials");
    if ((rc = t_launch(ctx, tb, false, d_tab, tab_cap, st))) return rc;
    uint64_t bytes = 0;
    for (auto& J : jobs)
      if (!J.done && J.blocks && !J.spec) bytes += (uint64_t)J.nbt * J.ba.box_cap * sizeof(T);
    ctx_span_end(ctx, ev, "tune_block_trials", bytes, st);
    for (auto& J : jobs)
      if ((rc = t_blocks_copy(J, st))) return rc;
  }
  if (join.on) {
    join.on = false;
    if ((rc = ctx_join(ctx, st))) return rc;
  }
  TCK(hipStreamSynchronize(st));
  for (auto& J : jobs) t_finish(J);
  ctx_prof_collect(ctx);
  return HPEZ_OK;
}

template <typename T>
int tune_group(hpez_ctx* ctx, const hpez_field_desc* d, const void* const* d_in,
               const hpez_tune_opts* o, hpez_config* cfg, uint8_t* const* h_bcfg,
               const uint64_t* bcap, const std::vector<int>& idx, int* rcs, hipStream_t st)
{
  std::vector<TJob<T>> jobs(idx.size());
  for (size_t k = 0; k < idx.size(); k++) {
    const int i = idx[k];
    jobs[k].d = &d[i];
    jobs[k].X = (const T*)d_in[i];
    jobs[k].o = &o[i];
    jobs[k].cfg = &cfg[i];
    jobs[k].h_bcfg = h_bcfg ? h_bcfg[i] : nullptr;
    jobs[k].bcap = bcap ? bcap[i] : 0;
  }
  const int rc = tune_jobs<T>(ctx, jobs, st);
  if (rc) return rc;
  for (size_t k = 0; k < idx.size(); k++) rcs[idx[k]] = jobs[k].rc;
  return HPEZ_OK;
}

}  // namespace

namespace hpez {
// the tuner's device bytes for a field with the default options
uint64_t tune_footprint(const hpez_field_desc* d, const hpez_config* c)
{
  hpez_tune_opts o;
  std::memset(&o, 0, sizeof o);
  o.global_rate = 0.01;
  o.sub_rate = 0.04;
  o.lorenzo_coef = 1.0;
  o.block_log2 = 5;
  o.block_wise = 1;
  o.allow_freeze = 1;
  o.allow_lorenzo = 1;
  hpez_config q = *c;
  uint8_t dummy = 0;
  TJob<float> J;  // sizes scale with the element size below
  J.d = d;
  J.o = &o;
  J.cfg = &q;
  J.h_bcfg = &dummy;
  J.bcap = ~0ull;
  t_init(J);
  const size_t s = d->dtype ? 8 : 4;
  J.scratch_bytes = trial_scratch(J.g, &o, s, J.gb.size(), J.gcap, J.nbt);
  return t_dev_bytes(J) + 2 * (3 * al256(2 * sizeof(TrialJob<double>)) + 3 * al256(3 * 8) + 512);
}
}  // namespace hpez

extern "C" int hpez_tune_batch(hpez_ctx* ctx, int n, const hpez_field_desc* desc,
                               const void* const* d_in, const hpez_tune_opts* opts,
                               hpez_config* out_cfg, uint8_t* const* h_block_cfg,
                               const uint64_t* block_cfg_cap, int* rcs, hipStream_t stream)
{
  if (!ctx || n < 0 || (n > 0 && (!desc || !d_in || !opts || !out_cfg || !rcs))) return HPEZ_EINVAL;
  for (int i = 0; i < n; i++) {
    if (!d_in[i]) return HPEZ_EINVAL;
    const int rc = check_desc(&desc[i]);
    if (rc) return rc;
  }
  if (!n) return HPEZ_OK;
  DeviceGuard dg(ctx_device(ctx));
  // integer fields: their values as float64 in the context's auxiliary buffer
  std::vector<const void*> in(d_in, d_in + n);
  size_t aux = 0;
  for (int i = 0; i < n; i++)
    if (dtype_int(desc[i].dtype)) aux += (points_of(&desc[i]) * 8 + 255) & ~(size_t)255;
  if (aux) {
    int arc = HPEZ_OK;
    uint8_t* p = (uint8_t*)ctx_aux(ctx, aux, &arc);
    if (arc) return arc;
    for (int i = 0; i < n; i++) {
      if (!dtype_int(desc[i].dtype)) continue;
      const uint64_t N = points_of(&desc[i]);
      if (launch_int_to_f64(in[i], desc[i].dtype, (double*)p, N, stream) != hipSuccess)
        return HPEZ_EDEVICE;
      in[i] = p;
      p += (N * 8 + 255) & ~(size_t)255;
    }
  }
  std::vector<int> f32, f64;
  for (int i = 0; i < n; i++) (desc[i].dtype == HPEZ_F32 ? f32 : f64).push_back(i);
  int rc = HPEZ_OK;
  if (!f32.empty())
    rc = tune_group<float>(ctx, desc, in.data(), opts, out_cfg, h_block_cfg, block_cfg_cap, f32,
                           rcs, stream);
  if (!rc && !f64.empty())
    rc = tune_group<double>(ctx, desc, in.data(), opts, out_cfg, h_block_cfg, block_cfg_cap, f64,
                            rcs, stream);
  if (rc) {
    ctx_drain(ctx, stream);
    return rc;
  }
  for (int i = 0; i < n; i++)
    if (rcs[i]) return rcs[i];
  return HPEZ_OK;
}

extern "C" int hpez_tune(hpez_ctx* ctx, const hpez_field_desc* desc, const void* d_in,
                         const hpez_tune_opts* opts, hpez_config* out_cfg, uint8_t* h_block_cfg,
                         uint64_t block_cfg_cap, hipStream_t stream)
{
  if (!ctx || !desc || !d_in || !opts || !out_cfg) return HPEZ_EINVAL;
  int rc1 = HPEZ_OK;
  const int rc =
      hpez_tune_batch(ctx, 1, desc, &d_in, opts, out_cfg, &h_block_cfg, &block_cfg_cap, &rc1, stream);
  return rc ? rc : rc1;
}
