// hpez_host.h -- host-side helpers of the runtime (stream layout, validation,
// Huffman codebook, geometry).  Not part of the public ABI.
#pragma once

#include <cstring>

#include <stdint.h>

#include <vector>

#include "block_dev.h"
#include "hpez_internal.h"

namespace hpez {

// Section sizes and offsets of one stream.
struct Layout {
  uint8_t predictor;  // 0 interpolation, 1 Lorenzo, 2 constant field
  double e;           // absolute error bound
  uint64_t n_blocks, n_anchor, n_unpred, n_outlier, n_patch, n_chunks, payload_bits;
  uint32_t sym_min, sym_max;
  uint64_t off_blocks, off_anchor, off_unpred, off_outl, off_pidx, off_pval, off_len, off_chunks,
      off_payload, total;
};

const char* err_text(int c);
uint64_t points_of(const hpez_field_desc* d);
int check_desc(const hpez_field_desc* d);
int check_cfg(const hpez_field_desc* d, const hpez_config* c, bool need_blocks);
uint64_t n_blocks(const hpez_field_desc* d, const hpez_config* c);
Geom make_geom(const hpez_field_desc* d, int frozen);
int n_active(const Geom& g);
Lattice make_lattice(const Geom& g, const int64_t* r, const int64_t* m);
double level_eb(double e, double alpha, double beta, int l);
uint64_t anchors_of(const Geom& g, int anchor_log2);
void layout(Layout* L, uint64_t s);
void write_header(uint8_t* h, const hpez_field_desc* d, const hpez_config* c, const Layout& L);
int read_header(const uint8_t* h, uint64_t n, hpez_field_desc* d, hpez_config* c, Layout* L);
int huffman_lengths(const uint32_t* hist, uint32_t nsym, uint8_t* len);
// device bytes of a tuning run with the default options (admission)
uint64_t tune_footprint(const hpez_field_desc* d, const hpez_config* c);
void canonical_codes(const uint8_t* len, uint32_t nsym, uint32_t* cw);
void canonical_codes_range(const uint8_t* len, uint32_t lo, uint32_t hi, uint32_t* cw);
void decode_tables_range(const uint8_t* len, uint32_t lo, uint32_t hi, uint32_t* lut,
                         uint16_t* sorted, uint64_t* lim, uint32_t* base);
// Canonical decoding tables: lut[2^kLutBits] (symbol << 8 | length, 0 for
// longer codes), symbols sorted by (length, symbol), and per length the window
// limit lim[l] and base[l] (kLmax + 1 entries each, index 0 unused).
void decode_tables(const uint8_t* len, uint32_t nsym, uint32_t* lut, uint16_t* sorted,
                   uint64_t* lim, uint32_t* base);
void md_table(const hpez_config* c, double* wq);

// Huffman payload (Sec. 4 step 4, api.cpp): encode codes[0, N) with the
// canonical codebook (h_len, h_cw: host, 2R entries; dlen, dcw: the same on the
// device) into the zeroed payload words and the per-chunk bit counts.  d_tab
// (2R words), d_flags (one word per chunk) and d_ticket are device scratch,
// h_tab (2R words) pinned host scratch.
int encode_payload(hpez_ctx* ctx, const uint16_t* code, uint64_t N, uint32_t chunk,
                   const uint8_t* h_len, const uint32_t* h_cw, uint32_t sym_min, uint32_t sym_max,
                   const uint8_t* dlen, const uint32_t* dcw, uint32_t* d_tab, uint32_t tab_words,
                   uint64_t* d_flags, uint32_t* d_ticket, uint32_t* h_tab, uint32_t* payload,
                   uint16_t* chunks, hipStream_t st);

// Lorenzo alternative (lorenzo.cpp): compress after the error bound is known
template <typename T>
int lorenzo_compress(hpez_ctx* ctx, const hpez_field_desc* d, const T* X, const hpez_config* c,
                     double e, uint8_t* out, uint64_t cap, uint64_t* out_size, hipStream_t st);

// fn(s) for every s in [lo, hi) with len[s] != 0, in increasing order; runs of
// zero lengths are skipped eight at a time (a code uses few of its symbols)
template <typename F>
inline void for_used(const uint8_t* len, uint32_t lo, uint32_t hi, F fn)
{
  uint32_t s = lo;
  for (; s < hi && (s & 7u); s++)
    if (len[s]) fn(s);
  for (; s + 8 <= hi; s += 8) {
    uint64_t w;
    std::memcpy(&w, len + s, 8);
    if (!w) continue;
    for (uint32_t j = 0; j < 8; j++)
      if (len[s + j]) fn(s + j);
  }
  for (; s < hi; s++)
    if (len[s]) fn(s);
}

// field types: integer fields run in double (the stream's anchors and
// verbatim values are double too); a negative 2e_l marks them for the kernels
inline bool dtype_int(int dt) { return dt >= HPEZ_U8; }
inline size_t dtype_size(int dt)
{
  return dt == HPEZ_F32 ? 4 : dt == HPEZ_F64 ? 8 : dt == HPEZ_U8 ? 1 : dt == HPEZ_I32 ? 4 : 2;
}
inline double twoe_of(double el, int dt) { return (dtype_int(dt) ? -2.0 : 2.0) * el; }
// values of integer field types to double and back (clamped), on the stream
hipError_t launch_int_to_f64(const void* in, int dt, double* out, uint64_t n, hipStream_t st);
hipError_t launch_f64_to_int(const double* in, int dt, void* out, uint64_t n, hipStream_t st);
// the context's auxiliary device buffer (integer fields' float64 copies),
// grown on demand, separate from the workspace
void* ctx_aux(hpez_ctx* c, size_t bytes, int* rc);

// Launch shapes chosen per context by hpez_autotune (measured on the device),
// keyed by kernel kind, dtype and the work's size class (floor log2 of its
// points or cells); the default applies until a shape is cached.  Shapes never
// change results, only speed.
enum TileKind { kTileFace = 0, kTileTrial = 1 };
uint32_t ctx_tile(hpez_ctx* c, int kind, int dtype, uint64_t work, uint32_t deflt);
// the cache's keys (kind << 16 | dtype << 8 | size class), for hpez_autotune:
// keys looked up since the last clear, a shape being tried for one key (value
// 0 removes it), and the chosen shape of a key
void ctx_tile_seen(hpez_ctx* c, bool clear, std::vector<uint64_t>* keys);
void ctx_tile_try(hpez_ctx* c, uint64_t key, uint32_t value);
void ctx_tile_set(hpez_ctx* c, uint64_t key, uint32_t value);
// face steps: lanes per work-group (64..256) and points per lane
inline uint32_t face_tile(uint32_t threads, uint32_t ppl) { return threads | ppl << 16; }
inline uint32_t face_threads(uint32_t t) { return t & 0xFFFFu; }
inline uint32_t face_ppl(uint32_t t) { return t >> 16; }

// context services (api.cpp)
void* ctx_ws(hpez_ctx* c, size_t bytes, int* rc);
uint8_t* ctx_pin(hpez_ctx* c, size_t bytes, int* rc);
// pinned staging of launch tables, reused by every call (synchronized between uses)
uint8_t* ctx_pin_tab(hpez_ctx* c, size_t bytes, int* rc);
int ctx_device(hpez_ctx* c);
// The context's second stream, made to wait for the work queued so far on st
// (nullptr on failure: the caller then queues everything on st).  ctx_join
// makes st wait for what was queued on the second stream since.
hipStream_t ctx_fork(hpez_ctx* c, hipStream_t st);
// A pool of up to four context streams for independent per-field work of a
// batch: ctx_fork_pool makes up to k of them wait for the work queued so far on
// st and returns how many (0: keep everything on st), or -1 when a HIP call
// failed; ctx_join_pool makes st wait for those k.
int ctx_fork_pool(hpez_ctx* c, hipStream_t st, int k, hipStream_t* out);
int ctx_join_pool(hpez_ctx* c, hipStream_t st, int k);
// after a call-level failure between launches: wait for the call's queued
// work on st, the second stream and the pool (staging may then be reused)
void ctx_drain(hpez_ctx* c, hipStream_t st);
int ctx_join(hpez_ctx* c, hipStream_t st);
// name: the group the span will close with (spans of other groups are not
// recorded while hpez_profile_only names one; a span opened without a name
// is then not recorded either)
hipEvent_t ctx_span_begin(hpez_ctx* c, hipStream_t st, const char* name = nullptr);
void ctx_span_end(hpez_ctx* c, hipEvent_t a, const char* name, uint64_t bytes, hipStream_t st);
void ctx_prof_collect(hpez_ctx* c);
// hpez_decompress on the device's fixed context: workspace `ws` (ws_bytes,
// device memory owned by the caller), static host staging, no second stream;
// requests beyond either give HPEZ_ENOMEM.  Calls on one device share it.
constexpr int kFixedDevices = 8;
int decompress_fixed(int device, void* ws, size_t ws_bytes, const void* d_in, uint64_t in_size,
                     void* d_out, uint64_t out_cap, hipStream_t stream);

// Scope guard that makes the context's device current.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev)
  {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard()
  {
    int cur = prev;
    if (hipGetDevice(&cur) != hipSuccess) return;
    if (prev >= 0 && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace hpez

namespace hpez {
// block-wise fast path (block.cpp)
template <typename T>
bool block_fast_ok(const hpez_config* c, const Geom& g);
template <typename T>
size_t block_fast_bytes(const Geom& g);

// One field's block phase: face arrays in `area` (block_fast_bytes), the face
// steps of every level below B, and the per-block kernel's arguments.
template <typename T>
struct BlockJobHost {
  // inputs
  const hpez_config* c = nullptr;
  Geom g;
  double e = 0;
  const T* X = nullptr;    // compress: the field
  bool xface = false;      // compress: family 2's face array prefilled with the field's values
  bool fcode2 = false;     // decompress: family 2's codes in f.code[2] (from the decoder)
  const T* Wg = nullptr;   // the grid holding anchors and levels >= B
  int dtype = 0;           // the field's type (integer fields: rounded reconstructions)
  uint16_t* code = nullptr;
  const uint8_t* d_bcfg = nullptr;
  const double* h_wq = nullptr;
  uint32_t* hist = nullptr;
  uint32_t hist_lo = 0;
  void* area = nullptr;
  T* out = nullptr;        // decompress: the field
  // built by block_job_prepare
  FaceGeo f;
  T* cval = nullptr;          // coarse levels' lattice values (in area)
  uint16_t* ccode = nullptr;  // coarse levels' lattice codes (in area)
  bool planes = false;        // coarse face levels in the plane kernel
  PlaneJob<T> pj[3];          // one per active family (wg_begin: the plane count)
  int npj = 0;
  size_t plane_lds = 0;
  BlockArgs ba;
  std::vector<FaceStep> steps[17];
  // per step its group: consecutive steps of a level with the same group are
  // independent (the odd sets of one multi-dimensional sub-step) and share a launch
  std::vector<int> sgrp[17];
  uint64_t nblocks = 0, npts = 0, face_pts = 0;
  size_t lds = 0;
};
template <typename T>
int block_job_prepare(hpez_ctx* ctx, BlockJobHost<T>& J);
// the face arrays' layout in a block phase area (block_fast_bytes)
template <typename T>
FaceGeo block_face_arrays(const Geom& g, void* area);
// device and pinned host bytes of the work tables of run_block_jobs
template <typename T>
size_t block_tables_bound(int n);  // any n jobs
template <typename T>
size_t block_jobs_table_bytes(const BlockJobHost<T>* jobs, int n);
// face phase then block phase of jobs [0, n) in fused launches (mode 0
// compress, 1 decompress); d_tables / h_tables: block_jobs_table_bytes each
template <typename T>
int run_block_jobs(hpez_ctx* ctx, BlockJobHost<T>* jobs, int n, int mode, void* d_tables,
                   uint8_t* h_tables, hipStream_t st);
}  // namespace hpez
