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

struct Work {
  TrialBox* boxes;
  void* scratch;
  size_t scratch_bytes;
  unsigned long long* score;
  unsigned long long* dummy;
  uint32_t* hist;
  int* flag;
  double* wq;
  unsigned long long* h_score;
  uint32_t* h_hist;
};

void fill_levels(TrialArgs& a, double e, const hpez_config* Q)
{
  for (int l = 1; l <= 16; l++) {
    const double el = level_eb(e, Q->alpha, Q->beta, l);
    a.el[l] = el;
    a.inv2e[l] = 1.0 / (2.0 * el);
    a.twoe[l] = 2.0 * el;
  }
  a.el[0] = a.inv2e[0] = a.twoe[0] = 0.0;
  double wq[3 * 16 * 4];
  md_table(Q, wq);
  for (int k = 0; k < 3; k++)
    for (int odd = 0; odd < 8; odd++)
      for (int d = 0; d < 4; d++) a.wmd[(k * 8 + odd) * 4 + d] = wq[(k * 16 + odd) * 4 + d];
}

template <typename T>
int global_tune(hpez_ctx* ctx, const hpez_field_desc* d, const T* X, const hpez_config* Q, double e,
                const hpez_tune_opts* o, int frozen, const hpez_interp* cand, Work& w,
                hpez_interp* level_out, double* H, hipStream_t st)
{
  const Geom g = make_geom(d, -1);
  const int Lb = o->block_log2;
  const int64_t B = (int64_t)1 << Lb;
  uint64_t cap;
  std::vector<TrialBox> bx = global_boxes(g, B, o->global_rate, &cap);
  const uint32_t nbx = (uint32_t)bx.size();
  const uint32_t nsym = 2 * Q->radius;
  if ((size_t)nbx * kNCand * cap * sizeof(T) > w.scratch_bytes &&
      cap * sizeof(T) > kTrialLdsBytes)
    return HPEZ_ENOMEM;
  TCK(hipMemcpyAsync(w.boxes, bx.data(), bx.size() * sizeof(TrialBox), hipMemcpyHostToDevice, st));
  TrialArgs a;
  std::memset(&a, 0, sizeof a);
  a.fg = g;
  a.frozen = frozen;
  a.L = Lb;
  a.R = Q->radius;
  a.box_cap = cap;
  a.max_ext = (int32_t)std::min<int64_t>(B + 1, INT32_MAX);
  a.score_mul = 4096.0 / e;
  fill_levels(a, e, Q);
  for (int i = 0; i < kNCand; i++) a.cand[i] = cand[i];
  TCK(hipMemsetAsync(w.score, 0, sizeof(unsigned long long) * kNCand * 16, st));
  hipEvent_t ev = ctx_span_begin(ctx, st);
  TCK(launch_trials<T>(a, w.boxes, nbx, kNCand, X, (T*)w.scratch, w.wq, w.score, nullptr, st));
  ctx_span_end(ctx, ev, "tune_trials", (uint64_t)nbx * cap * sizeof(T), st);
  TCK(hipMemcpyAsync(w.h_score, w.score, sizeof(unsigned long long) * kNCand * 16,
                     hipMemcpyDeviceToHost, st));
  TCK(hipStreamSynchronize(st));
  int best[17];
  for (int l = 1; l <= Lb; l++) {
    best[l] = 0;
    for (int ci = 1; ci < kNCand; ci++)
      if (w.h_score[ci * 16 + l - 1] < w.h_score[best[l] * 16 + l - 1]) best[l] = ci;
  }
  a.tuned = 1;
  a.hist_lo = trial_hist_lo(Q->radius);
  for (int l = 1; l <= Lb; l++) a.level[l - 1] = cand[best[l]];
  TCK(hipMemsetAsync(w.hist, 0, sizeof(uint32_t) * nsym, st));
  TCK(hipMemsetAsync(w.dummy, 0, sizeof(unsigned long long) * 16, st));
  TCK(launch_trials<T>(a, w.boxes, nbx, 1, X, (T*)w.scratch, w.wq, w.dummy, w.hist, st));
  TCK(hipMemcpyAsync(w.h_hist, w.hist, sizeof(uint32_t) * nsym, hipMemcpyDeviceToHost, st));
  TCK(hipStreamSynchronize(st));
  const int L = Q->anchor_log2;
  for (int l = 1; l <= 16; l++) {
    const int lb = l <= Lb ? l : Lb;
    level_out[l - 1] = l <= L ? cand[best[lb]] : cand[0];
  }
  const int64_t A = (int64_t)1 << Q->anchor_log2;
  *H = entropy_bits(w.h_hist, nsym) +
       (double)anchor_count(d, frozen, A) * (double)sizeof(T) * 8.0 / (double)points_of(d);
  return HPEZ_OK;
}

template <typename T>
int lorenzo_tune(const hpez_field_desc* d, const T* X, const hpez_config* Q, double e,
                 const hpez_tune_opts* o, Work& w, double* H, bool* supported, hipStream_t st)
{
  const Geom g = make_geom(d, -1);
  const int64_t B = (int64_t)1 << o->block_log2;
  uint64_t cap;
  std::vector<TrialBox> bx = global_boxes(g, B, o->global_rate, &cap);
  const uint32_t nsym = 2 * Q->radius;
  TCK(hipMemcpyAsync(w.boxes, bx.data(), bx.size() * sizeof(TrialBox), hipMemcpyHostToDevice, st));
  TCK(hipMemsetAsync(w.hist, 0, sizeof(uint32_t) * nsym, st));
  TCK(hipMemsetAsync(w.flag, 0, sizeof(int), st));
  TCK(launch_lorenzo_trial<T>(g, w.boxes, (uint32_t)bx.size(), (uint32_t)cap, X, 1.0 / (2.0 * e),
                              Q->radius, trial_hist_lo(Q->radius), w.hist, w.flag, st));
  int h_flag = 0;
  TCK(hipMemcpyAsync(w.h_hist, w.hist, sizeof(uint32_t) * nsym, hipMemcpyDeviceToHost, st));
  TCK(hipMemcpyAsync(&h_flag, w.flag, sizeof(int), hipMemcpyDeviceToHost, st));
  TCK(hipStreamSynchronize(st));
  *supported = h_flag == 0;
  *H = entropy_bits(w.h_hist, nsym);
  return HPEZ_OK;
}

template <typename T>
int block_tune(hpez_ctx* ctx, const hpez_field_desc* d, const T* X, const hpez_config* Q, double e,
               const hpez_tune_opts* o, int frozen, const hpez_interp* cand, Work& w,
               uint8_t* h_bcfg, hipStream_t st)
{
  const Geom g = make_geom(d, -1);
  const Geom gf = make_geom(d, frozen);
  const int64_t B = (int64_t)1 << o->block_log2;
  int64_t nb[4], nbt = 1;
  for (int k = 0; k < 4; k++) {
    nb[k] = (g.n[k] + B - 1) / B;
    nbt *= nb[k];
  }
  const int nact = n_active(gf);
  const int D = nact > 0 ? nact : 1;
  int64_t side = (int64_t)std::floor((double)B * std::pow(o->sub_rate, 1.0 / (double)D) + 0.5);
  if (side < 3) side = 3;
  if (side > B) side = B;
  int64_t As = 1;
  int al = 0;
  while (As * 2 <= side - 1) {
    As *= 2;
    al++;
  }
  std::vector<TrialBox> bx((size_t)nbt);
  uint64_t cap = 0;
  for (int64_t bi = 0; bi < nbt; bi++) {
    int64_t b[4];
    unravel(bi, nb, b);
    uint64_t pts = 1;
    for (int k = 0; k < 4; k++) {
      const int64_t ext = g.n[k] - b[k] * B < B ? g.n[k] - b[k] * B : B;
      bx[bi].m[k] = g.n[k] > 1 ? (side < ext ? side : ext) : 1;
      bx[bi].o[k] = b[k] * B + (ext - bx[bi].m[k]) / 2;
      pts *= (uint64_t)bx[bi].m[k];
    }
    cap = std::max(cap, pts);
  }
  if ((size_t)nbt * kNCand * cap * sizeof(T) > w.scratch_bytes && cap * sizeof(T) > kTrialLdsBytes)
    return HPEZ_ENOMEM;
  TCK(hipMemcpyAsync(w.boxes, bx.data(), bx.size() * sizeof(TrialBox), hipMemcpyHostToDevice, st));
  TrialArgs a;
  std::memset(&a, 0, sizeof a);
  a.fg = g;
  a.frozen = frozen;
  a.L = al;
  a.R = Q->radius;
  a.score_mode = 1;
  a.box_cap = cap;
  a.max_ext = (int32_t)side;
  a.score_mul = 4096.0 / e;
  fill_levels(a, e, Q);
  for (int i = 0; i < kNCand; i++) a.cand[i] = cand[i];
  hipEvent_t ev = ctx_span_begin(ctx, st);
  TCK(launch_trials<T>(a, w.boxes, (uint32_t)nbt, kNCand, X, (T*)w.scratch, w.wq, w.score, nullptr,
                       st));
  ctx_span_end(ctx, ev, "tune_block_trials", (uint64_t)nbt * cap * sizeof(T), st);
  std::vector<unsigned long long> h((size_t)nbt * kNCand);
  TCK(hipMemcpyAsync(h.data(), w.score, h.size() * sizeof(unsigned long long),
                     hipMemcpyDeviceToHost, st));
  TCK(hipStreamSynchronize(st));
  for (int64_t bi = 0; bi < nbt; bi++) {
    int besti = 0;
    for (int ci = 1; ci < kNCand; ci++)
      if (h[(size_t)bi * kNCand + ci] < h[(size_t)bi * kNCand + besti]) besti = ci;
    h_bcfg[bi] = (uint8_t)besti;
  }
  return HPEZ_OK;
}

template <typename T>
int tune_t(hpez_ctx* ctx, const hpez_field_desc* d, const T* X, const hpez_tune_opts* o,
           hpez_config* cfg, uint8_t* h_bcfg, uint64_t bcap, hipStream_t st)
{
  const uint64_t N = points_of(d);
  hpez_config Q;
  std::memset(&Q, 0, sizeof Q);
  Q.radius = cfg->radius;
  Q.chunk = cfg->chunk;
  Q.alpha = cfg->alpha;
  Q.beta = cfg->beta;
  Q.frozen_dim = -1;
  for (int k = 0; k < 3; k++)
    for (int j = 0; j < 4; j++) Q.md_w[k][j] = 1.0;
  for (int i = 0; i < 16; i++)
    for (int j = 0; j < 4; j++) {
      Q.level[i].order[j] = (uint8_t)j;
      Q.cand[i].order[j] = (uint8_t)j;
    }
  if (check_cfg(d, &Q, false)) return HPEZ_EINVAL;
  if (o->block_log2 < 1 || o->block_log2 > 8 || !(o->global_rate > 0) || !(o->sub_rate > 0) ||
      !(o->lorenzo_coef > 0))
    return HPEZ_EINVAL;
  int big = 0;
  for (int i = 0; i < d->ndims; i++) big += d->dims[i] > 1;
  Q.anchor_log2 = o->anchor_log2 ? o->anchor_log2 : (big >= 3 ? 6 : big == 2 ? 7 : 8);
  const Geom g = make_geom(d, -1);
  const int64_t B = (int64_t)1 << o->block_log2;
  int64_t nbt = 1;
  for (int k = 0; k < 4; k++) nbt *= (g.n[k] + B - 1) / B;
  if (o->block_wise && (!h_bcfg || bcap < (uint64_t)nbt)) return HPEZ_EINVAL;
  const uint32_t nsym = 2 * Q.radius;

  // workspace
  uint64_t gcap;
  const std::vector<TrialBox> gb = global_boxes(g, B, o->global_rate, &gcap);
  const size_t nbox = std::max((size_t)nbt, gb.size());
  size_t scratch = gcap * sizeof(T) > kTrialLdsBytes ? gb.size() * kNCand * gcap * sizeof(T) : 0;
  if (o->block_wise) {
    // largest sub-block: fewest active dims (one frozen) gives the longest side
    int big_dims = 0;
    for (int k = 0; k < 4; k++) big_dims += g.n[k] > 1;
    const int Dmin = n_active(g) > 1 ? n_active(g) - 1 : 1;
    int64_t side = (int64_t)std::floor((double)B * std::pow(o->sub_rate, 1.0 / (double)Dmin) + 0.5);
    side = std::min<int64_t>(std::max<int64_t>(side, 3), B);
    uint64_t bcap_pts = 1;
    for (int k = 0; k < big_dims; k++) bcap_pts *= (uint64_t)side;
    if (bcap_pts * sizeof(T) > kTrialLdsBytes)
      scratch = std::max(scratch, (size_t)nbt * kNCand * bcap_pts * sizeof(T));
  }
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t need = al(nbox * sizeof(TrialBox)) + al(scratch) +
                      al(nbox * kNCand * sizeof(unsigned long long)) + al(16 * 8) +
                      al(nsym * 4) + al(64) + al(3 * 16 * 4 * 8) + al(2 * 1024 * 8) + al(64) +
                      al(12 * 8);
  int rc;
  uint8_t* base = (uint8_t*)ctx_ws(ctx, need, &rc);
  if (rc) return rc;
  uint8_t* pin = ctx_pin(ctx, nsym * 4 + kNCand * 16 * 8 + 4096, &rc);
  if (rc) return rc;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    uint8_t* p = base + off;
    off += al(bytes);
    return p;
  };
  Work w;
  w.boxes = (TrialBox*)take(nbox * sizeof(TrialBox));
  w.scratch = take(scratch);
  w.scratch_bytes = scratch;
  w.score = (unsigned long long*)take(nbox * kNCand * sizeof(unsigned long long));
  w.dummy = (unsigned long long*)take(16 * 8);
  w.hist = (uint32_t*)take(nsym * 4);
  w.flag = (int*)take(64);
  w.wq = (double*)take(3 * 16 * 4 * 8);
  double* part = (double*)take(2 * 1024 * 8);
  double* mm = (double*)take(64);
  unsigned long long* sums = (unsigned long long*)take(12 * 8);
  w.h_hist = (uint32_t*)pin;
  w.h_score = (unsigned long long*)(pin + nsym * 4);
  double* h_mm = (double*)(pin + nsym * 4 + kNCand * 16 * 8);
  int* h_bad = (int*)(h_mm + 2);
  unsigned long long* h_sums = (unsigned long long*)(h_mm + 4);

  // error bound
  TCK(hipMemsetAsync(w.flag, 0, sizeof(int), st));
  TCK(launch_minmax<T>(X, N, part, w.flag, 1024, st));
  TCK(launch_minmax_final(part, 1024, mm, st));
  TCK(hipMemcpyAsync(h_mm, mm, 16, hipMemcpyDeviceToHost, st));
  TCK(hipMemcpyAsync(h_bad, w.flag, 4, hipMemcpyDeviceToHost, st));
  TCK(hipStreamSynchronize(st));
  if (*h_bad) return HPEZ_EINVAL;
  double e;
  bool constant = false;
  if (d->eb_mode == HPEZ_REL) {
    const double range = h_mm[1] - h_mm[0];
    if (range == 0) constant = true;
    e = d->eb * range;
  } else {
    e = d->eb;
  }
  hpez_interp cand[kNCand];
  candidate_list(d->ndims, cand);
  if (constant) {
    *cfg = Q;
    cfg->n_cand = 0;
    cfg->block_cfg = nullptr;
    for (int l = 0; l < 16; l++) cfg->level[l] = cand[0];
    return HPEZ_OK;
  }
  if (!(e > 0)) return HPEZ_EINVAL;

  // Sec. 6.1 statistics
  Geom gs = g;
  for (int k = 0; k < 4; k++)
    if (gs.act[k] && gs.n[k] < 8) gs.act[k] = 0;
  int any = 0;
  for (int k = 0; k < 4; k++) any |= gs.act[k];
  int64_t count = 0;
  std::memset(h_sums, 0, 12 * 8);
  if (any) {
    int64_t r[4], m[4];
    Lattice lat;
    lat.total = 1;
    for (int k = 0; k < 4; k++) {
      r[k] = gs.act[k] ? 4 : 0;
      m[k] = gs.act[k] ? 8 : 1;
      const int64_t hi = gs.act[k] ? gs.n[k] - 4 : gs.n[k] - 1;
      lat.first[k] = r[k];
      lat.step[k] = m[k];
      lat.cnt[k] = r[k] <= hi ? (uint32_t)((hi - r[k]) / m[k] + 1) : 0;
      lat.total *= lat.cnt[k];
    }
    count = (int64_t)lat.total;
    TCK(hipMemsetAsync(sums, 0, 12 * 8, st));
    hipEvent_t ev = ctx_span_begin(ctx, st);
    TCK(launch_stats<T>(X, gs, lat, 256.0 / e, sums, st));
    ctx_span_end(ctx, ev, "tune_stats", lat.total * (1 + 4 * n_active(gs)) * sizeof(T), st);
    TCK(hipMemcpyAsync(h_sums, sums, 12 * 8, hipMemcpyDeviceToHost, st));
    TCK(hipStreamSynchronize(st));
  }
  double sigma2[3][4];
  for (int k = 0; k < 3; k++)
    for (int j = 0; j < 4; j++) {
      const double s2 = count > 0 ? (double)h_sums[k * 4 + j] / (double)count : 1.0;
      sigma2[k][j] = s2;
      Q.md_w[k][j] = 1.0 / (s2 > 1.0 ? s2 : 1.0);
    }
  int fcand = -1;
  if (count > 0 && n_active(g) >= 2) {
    for (int k = 0; k < 4; k++)
      if (g.act[k] && g.n[k] >= 8 && (fcand < 0 || sigma2[0][k] > sigma2[0][fcand])) fcand = k;
  }
  double h_wq[3 * 16 * 4];
  md_table(&Q, h_wq);
  TCK(hipMemcpyAsync(w.wq, h_wq, sizeof h_wq, hipMemcpyHostToDevice, st));

  // Sec. 6.2 / 6.3
  hpez_interp lv[2][16];
  double H[2] = {0, 0};
  rc = global_tune<T>(ctx, d, X, &Q, e, o, -1, cand, w, lv[0], &H[0], st);
  if (rc) return rc;
  int frozen = -1;
  if (o->allow_freeze && fcand >= 0) {
    rc = global_tune<T>(ctx, d, X, &Q, e, o, fcand, cand, w, lv[1], &H[1], st);
    if (rc) return rc;
    if (H[1] < H[0]) frozen = fcand;
  }
  const double Hbest = frozen >= 0 ? H[1] : H[0];
  // Sec. 6.5
  bool lorenzo = false;
  if (o->allow_lorenzo) {
    double HL = 0;
    bool ok = true;
    rc = lorenzo_tune<T>(d, X, &Q, e, o, w, &HL, &ok, st);
    if (rc) return rc;
    if (ok && o->lorenzo_coef * HL < Hbest) lorenzo = true;
  }
  hpez_config out = Q;
  out.frozen_dim = (int8_t)(lorenzo ? -1 : frozen);
  out.predictor = lorenzo ? HPEZ_LORENZO : HPEZ_INTERP;
  for (int l = 0; l < 16; l++) out.level[l] = lv[frozen >= 0 ? 1 : 0][l];
  out.n_cand = 0;
  out.block_cfg = nullptr;
  // Sec. 6.6
  if (!lorenzo && o->block_wise) {
    rc = block_tune<T>(ctx, d, X, &Q, e, o, frozen, cand, w, h_bcfg, st);
    if (rc) return rc;
    out.block_log2 = o->block_log2;
    out.n_cand = kNCand;
    for (int i = 0; i < kNCand; i++) out.cand[i] = cand[i];
    out.block_cfg = h_bcfg;
  }
  ctx_prof_collect(ctx);
  *cfg = out;
  return HPEZ_OK;
}

}  // namespace

extern "C" int hpez_tune(hpez_ctx* ctx, const hpez_field_desc* desc, const void* d_in,
                         const hpez_tune_opts* opts, hpez_config* out_cfg, uint8_t* h_block_cfg,
                         uint64_t block_cfg_cap, hipStream_t stream)
{
  if (!ctx || !desc || !d_in || !opts || !out_cfg) return HPEZ_EINVAL;
  int rc = check_desc(desc);
  if (rc) return rc;
  DeviceGuard dg(ctx_device(ctx));
  if (desc->dtype == HPEZ_F32)
    return tune_t<float>(ctx, desc, (const float*)d_in, opts, out_cfg, h_block_cfg, block_cfg_cap,
                         stream);
  return tune_t<double>(ctx, desc, (const double*)d_in, opts, out_cfg, h_block_cfg, block_cfg_cap,
                        stream);
}
