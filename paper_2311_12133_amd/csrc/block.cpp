// block.cpp -- host orchestration of the block-wise fast path (k_block.hip):
// face arrays, the face phase of every level below B (global configuration),
// then one work-group per block for the interiors.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "block_dev.h"
#include "hpez_host.h"
#include "interp_dev.h"

namespace hpez {

#define BCK(x)                                  \
  do {                                          \
    if ((x) != hipSuccess) return HPEZ_EDEVICE; \
  } while (0)

constexpr size_t kLdsLimit = 160 * 1024;

// exact division multipliers for the kernels' index arithmetic (xmagic)
static void div_magic32(uint32_t d, uint32_t* m, int32_t* sh)
{
  const XDivisor x = xmagic(d);
  *m = x.m;
  *sh = x.sh;
}
constexpr size_t kPlaneLdsBytes = 150 * 1024;  // a plane lattice in the plane kernel

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
  // the coarse levels' lattice values and codes, kCoarseCells per block
  uint64_t nb = 1;
  for (int k = 0; k < 4; k++) nb *= (uint64_t)((g.n[k] + kBrick - 1) / kBrick);
  b += ((nb * kCoarseCells * sizeof(T) + 255) & ~(size_t)255) +
       ((nb * kCoarseCells * 2 + 255) & ~(size_t)255);
  return b;
}

// face steps of one job: levels below B (5 for B = 32), at most 15 steps each
constexpr size_t kMaxFaceSteps = kBrickLog2 * 15;

template <typename T>
size_t block_tables_bound(int n)
{
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t ent = kMaxFaceSteps * (size_t)n;
  return al(ent * sizeof(FaceEntry<T>)) + al((ent + kMaxFaceSteps) * 8) +
         al(n * sizeof(BlockJobDev<T>)) + al((n + 1) * 8) + 256 +
         al(3 * (size_t)n * sizeof(PlaneJob<T>)) + al((3 * (size_t)n + 1) * 8) + al((n + 1) * 8);
}

template <typename T>
FaceGeo block_face_arrays(const Geom& g, void* area)
{
  int64_t elems[4];
  FaceGeo f;
  face_geometry(g, kBrick, kBrickLog2, elems, &f);
  uint8_t* p = (uint8_t*)area;
  for (int k = 0; k < 4; k++) {
    if (!elems[k]) continue;
    f.val[k] = p;
    p += (elems[k] * sizeof(T) + 255) & ~(size_t)255;
    f.code[k] = (uint16_t*)p;
    p += (elems[k] * 2 + 255) & ~(size_t)255;
  }
  return f;
}

template <typename T>
int block_job_prepare(hpez_ctx* ctx, BlockJobHost<T>& J)
{
  (void)ctx;
  const Geom& g = J.g;
  const hpez_config* c = J.c;
  const int64_t B = kBrick;
  int64_t elems[4];
  face_geometry(g, B, kBrickLog2, elems, &J.f);
  J.f = block_face_arrays<T>(g, J.area);
  uint8_t* p = (uint8_t*)J.area;
  for (int k = 0; k < 4; k++) {
    if (!elems[k]) continue;
    p += (elems[k] * sizeof(T) + 255) & ~(size_t)255;
    p += (elems[k] * 2 + 255) & ~(size_t)255;
  }
  {
    uint64_t nb = 1;
    for (int k = 0; k < 4; k++) nb *= (uint64_t)((g.n[k] + kBrick - 1) / kBrick);
    J.cval = (T*)p;
    p += (nb * kCoarseCells * sizeof(T) + 255) & ~(size_t)255;
    J.ccode = (uint16_t*)p;
    p += (nb * kCoarseCells * 2 + 255) & ~(size_t)255;
  }
  const int Lb = c->block_log2;
  const int nact = n_active(g);
  int64_t r[4], m[4];
  J.face_pts = 0;
  for (int l = 0; l <= 16; l++) {
    J.steps[l].clear();
    J.sgrp[l].clear();
  }
  // coarse face levels on whole planes when every plane's lattice fits
  J.npj = 0;
  J.plane_lds = 0;
  J.planes = Lb > kCoarseL;
  for (int d = 0; d < 3 && J.planes; d++) {
    if (!g.act[d]) continue;
    int64_t E[3];
    for (int e = 0; e < 3; e++) E[e] = e == d ? 1 : (g.act[e] ? (g.n[e] - 1) / 4 + 1 : g.n[e]);
    const int64_t cells = E[0] * E[1] * E[2];
    // step row counts c1 * c2 stay within the division table: one of the
    // plane's active dims is halved in every step
    int64_t c12 = E[1] * E[2];
    if (d == 1) c12 = E[2];
    else if (d == 2) c12 = E[1];
    else {
      int64_t best = 0;
      if (g.act[1]) best = std::max(best, ((E[1] + 1) / 2) * E[2]);
      if (g.act[2]) best = std::max(best, E[1] * ((E[2] + 1) / 2));
      c12 = best;
    }
    if ((size_t)cells * sizeof(T) > kPlaneLdsBytes || c12 > (int64_t)kMagicMax ||
        E[0] > (int64_t)kMagicMax || E[1] > (int64_t)kMagicMax || E[2] > (int64_t)kMagicMax) {
      J.planes = false;
      break;
    }
    PlaneJob<T>& P = J.pj[J.npj++];
    std::memset(&P, 0, sizeof P);
    P.g = g;
    P.d = d;
    P.Ltop = Lb;
    for (int e = 0; e < 3; e++) P.E[e] = (int32_t)E[e];
    div_magic32((uint32_t)(E[1] * E[2]), &P.mg_b0, &P.sh_b0);
    div_magic32((uint32_t)E[2], &P.mg_e2, &P.sh_e2);
    P.R = c->radius;
    for (int l = 1; l <= 16; l++) {
      const double el = level_eb(J.e, c->alpha, c->beta, l);
      P.el_l[l] = el;
      P.inv2e_l[l] = 1.0 / (2.0 * el);
      P.twoe_l[l] = twoe_of(el, J.dtype);
    }
    for (int k = 0; k < 3; k++)
      for (int odd = 0; odd < 8; odd++)
        for (int e = 0; e < 4; e++) P.wmd[(k * 8 + odd) * 4 + e] = J.h_wq[(k * 16 + odd) * 4 + e];
    for (int l = 0; l < 16; l++) P.level[l] = c->level[l];
    P.wg_begin = (uint64_t)((g.n[d] - 1) / B + 1);  // planes (the launch offset is set later)
    J.plane_lds = std::max(J.plane_lds, (size_t)cells * sizeof(T));
  }
  if (!J.planes) J.npj = 0;
  for (int l = Lb; l >= 1; l--) {
    if (J.planes && l > kCoarseL) continue;
    const int64_t s = (int64_t)1 << (l - 1);
    const double el = level_eb(J.e, c->alpha, c->beta, l);
    const hpez_interp& ip = c->level[l - 1];
    FaceStep a;
    std::memset(&a, 0, sizeof a);
    a.g = g;
    a.kind = ip.kind;
    a.md = ip.md;
    a.s = s;
    a.el = el;
    a.inv2e = 1.0 / (2.0 * el);
    a.twoe = twoe_of(el, J.dtype);
    a.R = c->radius;
    // one step over every family whose planes the step touches; steps of one
    // group have no point in common and read none of each other's points
    int grp = 0;
    auto step = [&](const int64_t* rr, const int64_t* mm) {
      for (int k = 0; k < 4; k++) {
        a.first[k] = rr[k];
        a.step[k] = mm[k];
        a.cnt[k] = rr[k] <= g.n[k] - 1 ? (uint32_t)((g.n[k] - 1 - rr[k]) / mm[k] + 1) : 0;
        div_magic32(a.cnt[k], &a.mg[k], &a.msh[k]);
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
      J.face_pts += a.off[4];
      J.steps[l].push_back(a);
      J.sgrp[l].push_back(grp);
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
          for (int k = 0; k < 4; k++) a.wq[k] = J.h_wq[(ip.kind * 16 + odd) * 4 + k];
          if (ip.kind != 0 && ip.same_level) {
            // same-level cubic inside MD: the sub-step's checkerboard colour 0,
            // then colour 1 with the same-level stencils (a later group)
            for (int half = 0; half < 2; half++) {
              a.sl = half;
              a.mdhalf = 1 + half;
              grp = 2 * (cnt - 1) + half;
              step(r, m);
            }
            a.sl = 0;
            a.mdhalf = 0;
          } else {
            grp = cnt - 1;  // Sec. 5.4.1: one sub-step per number of odd coordinates
            step(r, m);
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
        a.odd = 0;
        // 1D passes (and their same-level halves) depend on each other
        if (ip.kind != 0 && ip.same_level) {
          m[pd] = 4 * s;
          r[pd] = s;
          a.sl = 0;
          grp = 2 * k;
          step(r, m);
          r[pd] = 3 * s;
          a.sl = 1;
          grp = 2 * k + 1;
          step(r, m);
          a.sl = 0;
        } else {
          a.sl = 0;
          grp = k;
          step(r, m);
        }
      }
    }
  }

  BlockArgs& ba = J.ba;
  std::memset(&ba, 0, sizeof ba);
  ba.g = g;
  J.nblocks = 1;
  J.npts = 1;
  for (int k = 0; k < 4; k++) {
    ba.nb[k] = (g.n[k] + B - 1) / B;
    J.nblocks *= (uint64_t)ba.nb[k];
    J.npts *= (uint64_t)g.n[k];
  }
  ba.L = Lb;
  ba.R = c->radius;
  ba.hist_lo = J.hist_lo;
  ba.vec = (g.n[2] % 4 == 0) && ((uintptr_t)J.X % 16 == 0) && ((uintptr_t)J.out % 16 == 0);
  for (int l = 1; l <= 16; l++) {
    const double el = level_eb(J.e, c->alpha, c->beta, l);
    ba.el_l[l] = el;
    ba.inv2e_l[l] = 1.0 / (2.0 * el);
    ba.twoe_l[l] = twoe_of(el, J.dtype);
  }
  for (uint32_t i = 0; i < c->n_cand && i < 16; i++) ba.cand[i] = c->cand[i];
  for (int k = 0; k < 3; k++)
    for (int odd = 0; odd < 8; odd++)
      for (int d = 0; d < 4; d++)
        ba.wmd[(k * 8 + odd) * 4 + d] = J.h_wq[(k * 16 + odd) * 4 + d];
  J.lds = block_lds_bytes<T>(g);
  return HPEZ_OK;
}

// face-step launch geometry of a step: work-groups of `per` points (lanes
// times points per lane; the kernel strides over the rest)
static uint64_t face_wgs(uint64_t pts, uint64_t per)
{
  uint64_t b = (pts + per - 1) / per;
  if (b > 65536) b = 65536;
  return b ? b : 1;
}

template <typename T>
size_t block_jobs_table_bytes(const BlockJobHost<T>* jobs, int n)
{
  size_t ent = 0, slots = 0;
  for (int l = 1; l <= 16; l++) {
    size_t mx = 0;
    for (int j = 0; j < n; j++) mx = std::max(mx, jobs[j].steps[l].size());
    slots += mx;
    for (int j = 0; j < n; j++) ent += jobs[j].steps[l].size();
  }
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  return al(ent * sizeof(FaceEntry<T>)) + al((ent + slots) * 8) + al(n * sizeof(BlockJobDev<T>)) +
         al((n + 1) * 8) + 256 + al(3 * (size_t)n * sizeof(PlaneJob<T>)) + al((3 * (size_t)n + 1) * 8) +
         al((n + 1) * 8);
}

template <typename T>
int run_block_jobs(hpez_ctx* ctx, BlockJobHost<T>* jobs, int n, int mode, void* d_tables,
                   uint8_t* h_tables, hipStream_t st)
{
  if (n <= 0) return HPEZ_OK;
  // anchors and levels >= B: copy the coarse grid into the face arrays
  for (int j = 0; j < n; j++) {
    BlockJobHost<T>& J = jobs[j];
    int64_t r[4], m[4];
    for (int k = 0; k < 4; k++) {
      r[k] = 0;
      m[k] = J.g.act[k] ? kBrick : 1;
    }
    const Lattice coarse = make_lattice(J.g, r, m);
    BCK(launch_face_init<T>(J.f, J.g, coarse, J.Wg, J.code, mode, st));
  }

  // every table of the launches below, built on the host and copied once
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  size_t ent = 0, slots = 0;
  int Lmax = 0;
  for (int l = 1; l <= 16; l++) {
    size_t mx = 0;
    for (int j = 0; j < n; j++) {
      mx = std::max(mx, jobs[j].steps[l].size());
      ent += jobs[j].steps[l].size();
    }
    slots += mx;
    if (mx) Lmax = l;
  }
  const size_t off_wg = al(ent * sizeof(FaceEntry<T>));
  const size_t off_jobs = off_wg + al((ent + slots) * 8);
  const size_t off_begin = off_jobs + al(n * sizeof(BlockJobDev<T>));
  const size_t off_planes = off_begin + al((n + 1) * 8);
  const size_t off_pwg = off_planes + al(3 * (size_t)n * sizeof(PlaneJob<T>));
  const size_t off_begin2 = off_pwg + al((3 * (size_t)n + 1) * 8);
  const size_t bytes = off_begin2 + al((n + 1) * 8);
  std::memset(h_tables, 0, bytes);
  FaceEntry<T>* he = (FaceEntry<T>*)h_tables;
  uint64_t* hw = (uint64_t*)(h_tables + off_wg);
  struct Launch {
    size_t e0, w0;
    int cnt;
    uint64_t wgs;
    bool narrow;
    uint32_t threads;
    int level;
  };
  std::vector<Launch> launches;
  size_t ei = 0, wi = 0;
  uint64_t face_pts = 0;
  for (int l = Lmax; l >= 1; l--) {
    // one launch per step group, over every job's steps of that group
    int ng = 0;
    for (int j = 0; j < n; j++)
      if (!jobs[j].sgrp[l].empty()) ng = std::max(ng, jobs[j].sgrp[l].back() + 1);
    for (int gi = 0; gi < ng; gi++) {
      // the launch shape for this launch's size class (hpez_autotune)
      uint64_t gpts = 0;
      for (int j = 0; j < n; j++)
        for (size_t k = 0; k < jobs[j].steps[l].size(); k++)
          if (jobs[j].sgrp[l][k] == gi) gpts += jobs[j].steps[l][k].off[4];
      const uint32_t tile =
          gpts ? ctx_tile(ctx, kTileFace, sizeof(T) == 4 ? 0 : 1, gpts, face_tile(256, 1))
               : face_tile(256, 1);
      Launch L{ei, wi, 0, 0, true, face_threads(tile), l};
      const uint64_t per = (uint64_t)face_threads(tile) * face_ppl(tile);
      for (int j = 0; j < n; j++)
      for (size_t k = 0; k < jobs[j].steps[l].size(); k++) {
        if (jobs[j].sgrp[l][k] != gi) continue;
        const FaceStep& a = jobs[j].steps[l][k];
        const uint64_t tot = a.off[4];
        if (!tot) continue;
        FaceEntry<T>& E = he[ei++];
        E.a = a;
        E.f = jobs[j].f;
        E.X = jobs[j].X;
        E.code = jobs[j].code;
        E.out = jobs[j].out;
        E.xface = jobs[j].xface ? 1 : 0;
        E.fcode2 = jobs[j].fcode2 ? 1 : 0;
        E.wg_begin = L.wgs;
        E.wg_count = face_wgs(tot, per);
        hw[wi++] = L.wgs;
        L.wgs += E.wg_count;
        L.narrow = L.narrow && tot < (1ull << 32);
        L.cnt++;
        face_pts += tot;
      }
      if (L.cnt) {
        hw[wi++] = L.wgs;  // end marker
        launches.push_back(L);
      }
    }
  }
  BlockJobDev<T>* hj = (BlockJobDev<T>*)(h_tables + off_jobs);
  uint64_t* hb = (uint64_t*)(h_tables + off_begin);
  uint64_t total_blocks = 0, npts = 0;
  // jobs whose box has at most two active dims (33 x 33 points or fewer) take
  // the 256-lane block kernel, several work-groups per CU; the table lists
  // them after the others, and begin2 rebases their block indices
  const size_t small_box = (((size_t)33 * 33 * sizeof(T) + 15) & ~(size_t)15) + (size_t)kBlockHistWin * 4;
  auto is_small = [&](const BlockJobHost<T>& J) {
    const int na = (int)J.g.act[0] + (int)J.g.act[1] + (int)J.g.act[2] + (int)J.g.act[3];
    return na <= 2 && J.lds <= small_box;
  };
  std::vector<int> perm;
  for (int pass = 0; pass < 2; pass++)
    for (int j = 0; j < n; j++)
      if (is_small(jobs[j]) == (pass == 1)) perm.push_back(j);
  int nbig = 0;
  while (nbig < n && !is_small(jobs[perm[nbig]])) nbig++;
  size_t lds = 0, lds_small = 0;
  for (int k = 0; k < n; k++) {
    const int j = perm[k];
    size_t& L = k < nbig ? lds : lds_small;
    L = std::max(L, jobs[j].lds);
    hj[k].a = jobs[j].ba;
    hj[k].f = jobs[j].f;
    hj[k].X = jobs[j].X;
    hj[k].code = jobs[j].code;
    hj[k].bcfg = jobs[j].d_bcfg;
    hj[k].hist = jobs[j].hist;
    hj[k].out = jobs[j].out;
    hj[k].cval = jobs[j].cval;
    hj[k].ccode = jobs[j].ccode;
    hj[k].block_begin = total_blocks;
    hb[k] = total_blocks;
    total_blocks += jobs[j].nblocks;
    npts += jobs[j].npts;
  }
  hb[n] = total_blocks;
  uint64_t* hb2 = (uint64_t*)(h_tables + off_begin2);
  for (int k = nbig; k <= n; k++) hb2[k - nbig] = hb[k] - hb[nbig];
  PlaneJob<T>* hp = (PlaneJob<T>*)(h_tables + off_planes);
  uint64_t* hpw = (uint64_t*)(h_tables + off_pwg);
  int np = 0;
  uint64_t plane_wgs = 0;
  size_t plane_lds = 0;
  for (int j = 0; j < n; j++) {
    for (int k = 0; k < jobs[j].npj; k++) {
      PlaneJob<T> P = jobs[j].pj[k];
      const uint64_t planes = P.wg_begin;
      P.f = jobs[j].f;
      P.X = jobs[j].X;
      P.code = jobs[j].code;
      P.out = jobs[j].out;
      P.wg_begin = plane_wgs;
      hp[np] = P;
      hpw[np] = plane_wgs;
      np++;
      plane_wgs += planes;
    }
    plane_lds = std::max(plane_lds, jobs[j].plane_lds);
  }
  hpw[np] = plane_wgs;
  uint8_t* dt = (uint8_t*)d_tables;
  BCK(hipMemcpyAsync(dt, h_tables, bytes, hipMemcpyHostToDevice, st));

  hipEvent_t ev = ctx_span_begin(ctx, st, mode == 0 ? "faces_predict" : "faces_reconstruct");
  BCK(launch_planes<T>((const PlaneJob<T>*)(dt + off_planes), (const uint64_t*)(dt + off_pwg), np,
                       plane_wgs, plane_lds, mode, st));
  // The coarse levels of every block on the block lattices need only the
  // face points of the coarse face levels (s >= 4): from the planes, or from
  // the face steps of those levels for fields whose planes do not fit, which
  // come first (launches run from the top level down).  The face steps of
  // levels 2 and 1 fill the other face points; they and the coarse levels
  // write disjoint arrays, so the coarse levels run on the second stream
  // beside them.
  auto face_launch = [&](const Launch& L) {
    return launch_face_steps<T>((const FaceEntry<T>*)dt + L.e0,
                                (const uint64_t*)(dt + off_wg) + L.w0, L.cnt, L.wgs, L.narrow,
                                mode, L.threads, st);
  };
  size_t li = 0;
  for (; li < launches.size() && launches[li].level > kCoarseL; li++)
    BCK(face_launch(launches[li]));
  hipStream_t cs = li == launches.size() ? st : ctx_fork(ctx, st);
  if (!cs) cs = st;
  hipEvent_t evc = ctx_span_begin(ctx, cs, mode == 0 ? "coarse_predict" : "coarse_reconstruct");
  BCK(launch_coarse_jobs<T>((const BlockJobDev<T>*)(dt + off_jobs), (const uint64_t*)(dt + off_begin),
                            n, total_blocks, mode, cs));
  ctx_span_end(ctx, evc, mode == 0 ? "coarse_predict" : "coarse_reconstruct",
               total_blocks * 729ull * (sizeof(T) + 2), cs);
  for (; li < launches.size(); li++) BCK(face_launch(launches[li]));
  ctx_span_end(ctx, ev, mode == 0 ? "faces_predict" : "faces_reconstruct",
               face_pts * (sizeof(T) + 2), st);
  if (cs != st) {
    const int rc = ctx_join(ctx, st);
    if (rc) return rc;
  }

  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx_device(ctx)) !=
          hipSuccess ||
      n_cu <= 0)
    return HPEZ_EDEVICE;
  ev = ctx_span_begin(ctx, st, mode == 0 ? "blocks_predict" : "blocks_reconstruct");
  if (nbig)
    BCK(launch_block_jobs<T>((const BlockJobDev<T>*)(dt + off_jobs), (const uint64_t*)(dt + off_begin),
                             nbig, hb[nbig], lds, n_cu, mode, false, st));
  if (nbig < n)
    BCK(launch_block_jobs<T>((const BlockJobDev<T>*)(dt + off_jobs) + nbig,
                             (const uint64_t*)(dt + off_begin2), n - nbig, hb[n] - hb[nbig],
                             lds_small, n_cu, mode, true, st));
  ctx_span_end(ctx, ev, mode == 0 ? "blocks_predict" : "blocks_reconstruct",
               npts * (sizeof(T) + 2), st);
  return HPEZ_OK;
}

#define INST(T)                                                                                  \
  template bool block_fast_ok<T>(const hpez_config*, const Geom&);                               \
  template size_t block_fast_bytes<T>(const Geom&);                                              \
  template size_t block_tables_bound<T>(int);                                                    \
  template int block_job_prepare<T>(hpez_ctx*, BlockJobHost<T>&);                                \
  template FaceGeo block_face_arrays<T>(const Geom&, void*);                                    \
  template size_t block_jobs_table_bytes<T>(const BlockJobHost<T>*, int);                        \
  template int run_block_jobs<T>(hpez_ctx*, BlockJobHost<T>*, int, int, void*, uint8_t*,         \
                                 hipStream_t);
INST(float)
INST(double)

}  // namespace hpez
