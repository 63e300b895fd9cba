// autotune.cpp -- hpez_autotune: launch shapes measured on the device for a
// field, cached in the context (no effect on any result, only on speed).
//
// Two shapes are tuned: the face steps' lanes per work-group and points per
// lane (3 x 4 candidates per launch size class), and the lanes per work-group
// of the tuner's region trials (64, 256, 1024 per region size class).  For
// each size class the field's own calls use, every candidate is tried while
// the other classes keep their current shapes; the candidate with the least
// time of its kernel group (the sum over a compress + decompress, resp. a
// tune; best of three repetitions after one warm-up) is cached.
#include <algorithm>
#include <cstring>
#include <vector>

#include "hpez_host.h"
#include "hpez_internal.h"

namespace hpez {
namespace {

// kernel-group time (ms) of the last profiled call(s): groups whose name
// starts with one of `prefixes`
double group_ms(hpez_ctx* ctx, const char* const* prefixes, int np)
{
  hpez_kernel_stat st[64];
  int n = 0;
  if (hpez_profile_read(ctx, st, 64, &n)) return 1e30;
  double ms = 0.0;
  for (int i = 0; i < n && i < 64; i++)
    for (int p = 0; p < np; p++)
      if (std::strncmp(st[i].name, prefixes[p], std::strlen(prefixes[p])) == 0) ms += st[i].total_ms;
  return ms;
}

struct Runner {
  hpez_ctx* ctx;
  const hpez_field_desc* d;
  const void* x;
  const hpez_config* cfg;
  const hpez_tune_opts* topts;
  void* z = nullptr;
  void* xr = nullptr;
  uint64_t cap = 0, xbytes = 0;
  std::vector<uint8_t> bcfg;
  hipStream_t st;

  // one compress + decompress (faces) or one tune (trials); rc on failure
  int run(int what)
  {
    if (what == kTileFace) {
      uint64_t size = 0;
      int rc = hpez_compress(ctx, d, x, cfg, z, cap, &size, st);
      if (!rc) rc = hpez_decompress(ctx, z, size, xr, xbytes, st);
      return rc;
    }
    hpez_config out = *cfg;
    return hpez_tune(ctx, d, x, topts, &out, bcfg.data(), bcfg.size(), st);
  }

  // best-of-three time of the group after one warm-up, under the current shapes
  int time(int what, double* ms)
  {
    static const char* face[] = {"faces_"};
    static const char* trial[] = {"tune_trials", "tune_block_trials", "tune_ab_trials"};
    int rc = run(what);
    if (rc) return rc;
    *ms = 1e30;
    for (int r = 0; r < 3; r++) {
      hpez_profile_enable(ctx, 1);
      rc = run(what);
      const double t = what == kTileFace ? group_ms(ctx, face, 1) : group_ms(ctx, trial, 3);
      hpez_profile_enable(ctx, 0);
      if (rc) return rc;
      *ms = std::min(*ms, t);
    }
    return HPEZ_OK;
  }
};

int tune_kind(Runner& R, int what, hpez_tile_choice* out, int cap, int* n)
{
  std::vector<uint64_t> keys;
  ctx_tile_seen(R.ctx, true, nullptr);
  int rc = R.run(what);
  if (rc) return rc;
  ctx_tile_seen(R.ctx, true, &keys);
  std::vector<uint32_t> cands;
  if (what == kTileFace) {
    for (uint32_t t : {64u, 128u, 256u})
      for (uint32_t p : {1u, 2u, 4u, 8u}) cands.push_back(face_tile(t, p));
  } else {
    cands = {64u, 256u, 1024u};
  }
  for (uint64_t k : keys) {
    if ((int)(k >> 16) != what) continue;
    double best = 1e30, base = 0.0;
    uint32_t pick = 0;
    for (uint32_t c : cands) {
      ctx_tile_try(R.ctx, k, c);
      double ms = 0.0;
      rc = R.time(what, &ms);
      if (rc) break;
      if (ms < best) {
        best = ms;
        pick = c;
      }
    }
    ctx_tile_try(R.ctx, k, 0);
    if (rc) return rc;
    // the time under the shape the key had before (cached or default)
    rc = R.time(what, &base);
    if (rc) return rc;
    ctx_tile_set(R.ctx, k, pick);
    if (*n < cap) {
      hpez_tile_choice& o = out[*n];
      o.kind = what;
      o.dtype = (int32_t)(k >> 8 & 0xFF);
      o.size_class = (int32_t)(k & 0xFF);
      o.value = pick;
      o.ms_before = base;
      o.ms_best = best;
    }
    (*n)++;
  }
  return HPEZ_OK;
}

}  // namespace
}  // namespace hpez

using namespace hpez;

extern "C" int hpez_autotune(hpez_ctx* ctx, const hpez_field_desc* desc, const void* d_in,
                             const hpez_config* cfg, const hpez_tune_opts* topts,
                             hpez_tile_choice* out, int cap, int* n_out, hipStream_t stream)
{
  if (!ctx || !desc || !d_in || !cfg || !n_out || cap < 0 || (cap > 0 && !out)) return HPEZ_EINVAL;
  int rc = check_desc(desc);
  if (rc) return rc;
  *n_out = 0;
  Runner R{ctx, desc, d_in, cfg, topts};
  R.st = stream;
  rc = hpez_compress_bound(desc, cfg, &R.cap);
  if (rc) return rc;
  R.xbytes = points_of(desc) * dtype_size(desc->dtype);
  if (topts) {
    uint64_t nb = 1;
    const uint64_t B = (uint64_t)1 << (topts->block_log2 ? topts->block_log2 : 5);
    for (int i = 0; i < desc->ndims; i++) nb *= (desc->dims[i] + B - 1) / B;
    R.bcfg.assign(nb, 0);
  }
  if (hipMalloc(&R.z, R.cap) != hipSuccess) return HPEZ_ENOMEM;
  if (hipMalloc(&R.xr, R.xbytes) != hipSuccess) {
    (void)hipFree(R.z);
    return HPEZ_ENOMEM;
  }
  rc = tune_kind(R, kTileFace, out, cap, n_out);
  if (!rc && topts) rc = tune_kind(R, kTileTrial, out, cap, n_out);
  (void)hipFree(R.z);
  (void)hipFree(R.xr);
  return rc;
}
