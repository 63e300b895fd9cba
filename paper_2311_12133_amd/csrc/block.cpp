// block.cpp -- host orchestration of the block-wise fast path (k_block.hip):
// face arrays, the face phase of every level below B (global configuration),
// then one work-group per block for the interiors.

#include <hip/hip_runtime.h>

#include <cstring>

#include "block_dev.h"
#include "hpez_host.h"
#include "interp_dev.h"

namespace hpez {

#define BCK(x)                                  \
  do {                                          \
    if ((x) != hipSuccess) return HPEZ_EDEVICE; \
  } while (0)

constexpr size_t kLdsLimit = 160 * 1024;

template <typename T>
bool block_fast_ok(const hpez_config* c, const Geom& g)
{
  if (c->block_log2 != kBrickLog2 || c->anchor_log2 < c->block_log2) return false;
  if (g.n[3] != 1) return false;  // up to three dims
  return block_lds_bytes<T>(g) <= kLdsLimit;
}

static void face_geometry(const Geom& g, int64_t B, int blog2, int64_t* elems, FaceGeo* f)
{
  std::memset(f, 0, sizeof *f);
  f->B = B;
  f->blog2 = blog2;
  for (int e = 0; e < 4; e++) {
    if (!g.act[e]) {
      elems[e] = 0;
      continue;
    }
    int64_t plane = 1;
    for (int k = 0; k < 4; k++)
      if (k != e) plane *= g.n[k];
    int64_t st = 1;
    for (int k = 3; k >= 0; k--) {
      if (k == e) continue;
      f->fs[e][k] = st;
      st *= g.n[k];
    }
    f->plane[e] = plane;
    elems[e] = ((g.n[e] - 1) / B + 1) * plane;
  }
}

template <typename T>
size_t block_fast_bytes(const Geom& g)
{
  int64_t elems[4];
  FaceGeo f;
  face_geometry(g, kBrick, kBrickLog2, elems, &f);
  size_t b = 0;
  for (int e = 0; e < 4; e++)
    b += ((elems[e] * sizeof(T) + 255) & ~(size_t)255) + ((elems[e] * 2 + 255) & ~(size_t)255);
  return b + 1024;  // + the work counter of the block kernel
}

template <typename T>
int run_block_fast(hpez_ctx* ctx, const hpez_config* c, const Geom& g, double e, const T* X,
                   const T* Wg, uint16_t* code, const uint8_t* d_bcfg, const double* d_wq,
                   const double* h_wq, uint32_t* hist, uint32_t hist_lo, void* area, T* out,
                   int mode, hipStream_t st)
{
  const int64_t B = kBrick;
  int64_t elems[4];
  FaceGeo f;
  face_geometry(g, B, kBrickLog2, elems, &f);
  uint8_t* p = (uint8_t*)area;
  for (int k = 0; k < 4; k++) {
    if (!elems[k]) continue;
    f.val[k] = p;
    p += (elems[k] * sizeof(T) + 255) & ~(size_t)255;
    f.code[k] = (uint16_t*)p;
    p += (elems[k] * 2 + 255) & ~(size_t)255;
  }
  uint32_t* ticket = (uint32_t*)p;
  // anchors and levels >= B: copy the coarse grid into the face arrays
  int64_t r[4], m[4];
  for (int k = 0; k < 4; k++) {
    r[k] = 0;
    m[k] = g.act[k] ? B : 1;
  }
  const Lattice coarse = make_lattice(g, r, m);
  BCK(launch_face_init<T>(f, g, coarse, Wg, code, mode, st));

  const int Lb = c->block_log2;
  const int nact = n_active(g);
  hipEvent_t ev = ctx_span_begin(ctx, st);
  uint64_t face_pts = 0;
  for (int l = Lb; l >= 1; l--) {
    const int64_t s = (int64_t)1 << (l - 1);
    const double el = level_eb(e, c->alpha, c->beta, l);
    const hpez_interp& ip = c->level[l - 1];
    FaceStep a;
    std::memset(&a, 0, sizeof a);
    a.g = g;
    a.kind = ip.kind;
    a.md = ip.md;
    a.s = s;
    a.el = el;
    a.inv2e = 1.0 / (2.0 * el);
    a.twoe = 2.0 * el;
    a.R = c->radius;
    // one launch per step over every family whose planes the step touches
    auto step = [&](const int64_t* rr, const int64_t* mm) -> int {
      for (int k = 0; k < 4; k++) {
        a.first[k] = rr[k];
        a.step[k] = mm[k];
        a.cnt[k] = rr[k] <= g.n[k] - 1 ? (uint32_t)((g.n[k] - 1 - rr[k]) / mm[k] + 1) : 0;
      }
      a.off[0] = 0;
      for (int d = 0; d < 4; d++) {
        // a step that predicts odd multiples of s along d has no points on d's planes
        uint64_t tot = 0;
        if (g.act[d] && rr[d] == 0) {
          tot = (uint64_t)((g.n[d] - 1) / B + 1);
          for (int k = 0; k < 4; k++)
            if (k != d) tot *= a.cnt[k];
        }
        a.off[d + 1] = a.off[d] + tot;
      }
      face_pts += a.off[4];
      if (launch_face_step<T>(a, f, X, code, out, mode, st) != hipSuccess) return HPEZ_EDEVICE;
      return HPEZ_OK;
    };
    if (ip.md) {
      for (int cnt = 1; cnt <= nact; cnt++)
        for (unsigned odd = 1; odd < 16; odd++) {
          bool ok = (int)__builtin_popcount(odd) == cnt;
          for (int k = 0; k < 4; k++)
            if ((odd >> k & 1u) && !g.act[k]) ok = false;
          if (!ok) continue;
          for (int k = 0; k < 4; k++) {
            if (!g.act[k]) { r[k] = 0; m[k] = 1; }
            else if (odd >> k & 1u) { r[k] = s; m[k] = 2 * s; }
            else { r[k] = 0; m[k] = 2 * s; }
          }
          a.odd = odd;
          for (int k = 0; k < 4; k++) a.wq[k] = h_wq[(ip.kind * 16 + odd) * 4 + k];
          int rc = step(r, m);
          if (rc) return rc;
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
        a.odd = 0;
        if (ip.kind != 0 && ip.same_level) {
          m[pd] = 4 * s;
          r[pd] = s;
          a.sl = 0;
          int rc = step(r, m);
          if (rc) return rc;
          r[pd] = 3 * s;
          a.sl = 1;
          rc = step(r, m);
          if (rc) return rc;
          a.sl = 0;
        } else {
          a.sl = 0;
          int rc = step(r, m);
          if (rc) return rc;
        }
      }
    }
  }
  ctx_span_end(ctx, ev, mode == 0 ? "faces_predict" : "faces_reconstruct",
               face_pts * (sizeof(T) + 2), st);

  BlockArgs ba;
  std::memset(&ba, 0, sizeof ba);
  ba.g = g;
  uint64_t npts = 1;
  for (int k = 0; k < 4; k++) {
    ba.nb[k] = (g.n[k] + B - 1) / B;
    npts *= (uint64_t)g.n[k];
  }
  ba.L = Lb;
  ba.R = c->radius;
  ba.hist_lo = hist_lo;
  ba.vec = (g.n[2] % 4 == 0) && ((uintptr_t)X % 16 == 0) && ((uintptr_t)out % 16 == 0);
  for (int l = 1; l <= 16; l++) {
    const double el = level_eb(e, c->alpha, c->beta, l);
    ba.el_l[l] = el;
    ba.inv2e_l[l] = 1.0 / (2.0 * el);
    ba.twoe_l[l] = 2.0 * el;
  }
  for (uint32_t i = 0; i < c->n_cand && i < 16; i++) ba.cand[i] = c->cand[i];
  for (int k = 0; k < 3; k++)
    for (int odd = 0; odd < 8; odd++)
      for (int d = 0; d < 4; d++) ba.wmd[(k * 8 + odd) * 4 + d] = h_wq[(k * 16 + odd) * 4 + d];
  ev = ctx_span_begin(ctx, st);
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx_device(ctx)) !=
          hipSuccess ||
      n_cu <= 0)
    return HPEZ_EDEVICE;
  BCK(hipMemsetAsync(ticket, 0, sizeof(uint32_t), st));
  BCK(launch_blocks<T>(ba, f, X, code, d_bcfg, hist, out, ticket, n_cu, mode, st));
  ctx_span_end(ctx, ev, mode == 0 ? "blocks_predict" : "blocks_reconstruct",
               npts * (sizeof(T) + 2), st);
  return HPEZ_OK;
}

#define INST(T)                                                                                  \
  template bool block_fast_ok<T>(const hpez_config*, const Geom&);                               \
  template size_t block_fast_bytes<T>(const Geom&);                                              \
  template int run_block_fast<T>(hpez_ctx*, const hpez_config*, const Geom&, double, const T*,   \
                                 const T*, uint16_t*, const uint8_t*, const double*,             \
                                 const double*, uint32_t*, uint32_t, void*, T*, int, hipStream_t);
INST(float)
INST(double)

}  // namespace hpez
