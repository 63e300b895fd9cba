/*
 * hpez.h -- C ABI of the MI355X HPEZ compression library.
 *
 * The library implements the data-parallel hot path of HPEZ (Liu et al.,
 * "High-performance Effective Scientific Error-bounded Lossy Compression with
 * Auto-tuned Multi-component Interpolation", SIGMOD 2024) as HIP kernels for
 * gfx950:
 *   - compression C_theta(X) -> Z and decompression D_theta(Z) -> X' under
 *     the point-wise bound |x - x'| <= e of Sec. 3.1, Eq. (1);
 *   - the level-wise interpolation predictor of Sec. 5 with linear-scale
 *     quantization (Sec. 4, step 3) and Huffman coding (Sec. 4, step 4);
 *   - the auto-tuner of Sec. 6.
 *
 * Conventions for every entry point:
 *   - Device pointers ("d_") are memory on the context's GPU (for instance
 *     torch tensors' data_ptr()); host pointers ("h_" or unprefixed structs) are
 *     ordinary process memory.  The caller owns every buffer it passes; the
 *     library keeps no pointer past the call (except a decompression plan,
 *     which borrows its streams and outputs while it lives).
 *   - `stream` is a hipStream_t (NULL = the default stream) on which all
 *     device work of the call is ordered.  Calls that need a result on the host
 *     (compress: the stream size; tune: the decisions) synchronise that stream
 *     before returning; all other calls return after enqueueing.
 *   - Return value: HPEZ_OK (0) or a negative error code; hpez_strerror()
 *     describes it.  No exception crosses the ABI.  After HPEZ_EDEVICE the
 *     context should be destroyed.
 *   - A context is used by one host thread at a time.
 *
 * Arrays are row-major with the last dimension varying fastest.
 */
#ifndef HPEZ_H
#define HPEZ_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HPEZ_OK = 0,
  HPEZ_EINVAL = -1,      /* invalid argument, shape, bound, configuration, or non-finite input */
  HPEZ_ENOMEM = -2,      /* device or host allocation failed */
  HPEZ_EDEVICE = -3,     /* a HIP call failed */
  HPEZ_ECORRUPT = -4,    /* the compressed stream is malformed */
  HPEZ_ENOSPC = -5,      /* output capacity too small */
  HPEZ_EUNSUPPORTED = -6 /* valid request this build does not handle */
};

/* Field types.  Integer fields (the paper's integer datasets) run the method in
 * float64 on their values, each rebuilt value rounded to the nearest integer
 * (ties to even) before the bound check, and are reconstructed in their own
 * type (clamped to its range, which keeps the bound); their streams store
 * anchors and verbatim values as float64.  They use the interpolation
 * predictor only (HPEZ_LORENZO gives HPEZ_EUNSUPPORTED; the tuner does not try
 * it). */
enum { HPEZ_F32 = 0, HPEZ_F64 = 1, HPEZ_U8 = 2, HPEZ_U16 = 3, HPEZ_I16 = 4, HPEZ_I32 = 5 };
enum { HPEZ_ABS = 0, HPEZ_REL = 1 };
enum { HPEZ_INTERP = 0, HPEZ_LORENZO = 1 };
enum { HPEZ_LINEAR = 0, HPEZ_CUBIC_NAK = 1, HPEZ_CUBIC_NATURAL = 2 };

/* One interpolation configuration (the choices tuned per level in Sec. 6.2):
 *   kind        0 linear spline Eq. (2), 1 not-a-knot cubic Eq. (6),
 *               2 natural cubic Eq. (8);
 *   md          0: one dimension at a time (1D style); 1: multi-dimensional
 *               interpolation, Eq. (9), Sec. 5.3;
 *   same_level  cubic: split every pass (1D style: points at s, then 3s mod 4s
 *               along the pass dim) or every multi-dimensional sub-step
 *               (checkerboard colour 0, then 1: the parity of the sum over the
 *               odd dims of (x_d - s) / 2s) in two, the second half using the
 *               same-level stencils Eq. (13)/(14), Sec. 5.4.2;
 *   order       1D style: the dimension of each pass, first pass first; the
 *               first ndims entries must be a permutation of 0..ndims-1. */
typedef struct {
  uint8_t kind;
  uint8_t md;
  uint8_t same_level;
  uint8_t order[4];
  uint8_t pad;
} hpez_interp;

/* The field: dtype (HPEZ_F32 ... HPEZ_I32), 1..4 dims (row-major), and the error
 * bound: absolute (eb = e) or value-range relative (e = eb * (max - min),
 * Sec. 7.1.3).  eb > 0 and finite.  The product of dims must be below 2^32. */
typedef struct {
  uint8_t dtype;
  uint8_t ndims;
  uint8_t eb_mode;
  uint8_t pad[5];
  uint64_t dims[4];
  double eb;
} hpez_field_desc;

/* Predictor configuration (theta of Eq. 1).
 *   predictor    HPEZ_INTERP, or HPEZ_LORENZO (first-order Lorenzo, Sec. 6.5);
 *   anchor_log2  anchor stride A = 2^anchor_log2 (Sec. 5.1), 0..16;
 *   block_log2   0, or block side B = 2^block_log2 for block-wise configurations
 *                (Sec. 6.6): levels with stride < B use, per block,
 *                cand[block_cfg[b]];
 *   frozen_dim   -1, or a dimension that is never interpolated along (Sec. 6.3);
 *   radius       quantization radius R (1..32768): codes are q + R, 0 marks a
 *                value stored verbatim;
 *   chunk        Huffman chunk length in symbols (power of two, 64..1024);
 *   alpha, beta  level error bounds e_l = e / min(alpha^(l-1), beta), Eq. (15),
 *                both >= 1;
 *   md_w         per stencil kind and dimension, the weight 1/sigma^2 of Eq. (12)
 *                used by multi-dimensional interpolation (> 0);
 *   level        level[l-1] is the configuration of level l (stride 2^(l-1));
 *   cand, n_cand block-wise candidates;
 *   block_cfg    host array of one candidate index per block (blocks in
 *                row-major order, ceil(dims[d] / B) per dim), or NULL when
 *                block_log2 == 0.  Borrowed for the call. */
typedef struct {
  uint8_t predictor;
  uint8_t anchor_log2;
  uint8_t block_log2;
  int8_t frozen_dim;
  uint32_t radius;
  uint32_t chunk;
  uint32_t n_cand;
  double alpha;
  double beta;
  double md_w[3][4];
  hpez_interp level[16];
  hpez_interp cand[16];
  const uint8_t* block_cfg;
} hpez_config;

/* Options of the auto-tuner (Sec. 6).
 *   global_rate  fraction of B^D blocks whose (B+1)^D boxes feed global tuning;
 *   sub_rate     volume fraction of the centred sub-block of block-wise tuning
 *                (the paper's default is 0.04);
 *   lorenzo_coef multiplies the Lorenzo bit-rate estimate (Sec. 6.5);
 *   block_log2   tuning block side (the paper uses 32, i.e. 5);
 *   allow_freeze, allow_lorenzo, block_wise  enable Sec. 6.3 / 6.5 / 6.6;
 *   anchor_log2  0 for the default (64 for 3+ dims, 128 for 2, 256 for 1);
 *   tune_ab      tune the level-wise bound of Eq. (15) (Sec. 6.4): when the
 *                interpolation predictor is kept, the tuned configuration is
 *                run on the global regions under each (alpha, beta) of the grid
 *                (1, 1), {1.25, 1.5, 1.75, 2} x {1.5, 2, 3, 4}, and the pair with
 *                the best rate-distortion score (quality in dB against e minus
 *                20 log10(2) dB per estimated bit) is returned in out_cfg and
 *                used by the block-wise trials; otherwise the caller's alpha and
 *                beta are kept. */
typedef struct {
  double global_rate;
  double sub_rate;
  double lorenzo_coef;
  uint8_t block_log2;
  uint8_t allow_freeze;
  uint8_t allow_lorenzo;
  uint8_t block_wise;
  uint8_t anchor_log2;
  uint8_t tune_ab;
  uint8_t pad[2];
} hpez_tune_opts;

typedef struct hpez_ctx hpez_ctx;

/* Human-readable text for an error code.  Static storage. */
const char* hpez_strerror(int code);

/* Create a context bound to GPU `device`; it owns a growable device workspace
 * and the per-device scratch state.  On first use it also creates a second
 * HIP stream (default priority) for work that can overlap the caller's
 * stream; that work is forked from and joined back to the caller's stream with
 * events inside each call, so ordering on the caller's stream is as if
 * everything ran there.  Destroy releases everything. */
int hpez_ctx_create(hpez_ctx** out, int device);
void hpez_ctx_destroy(hpez_ctx* ctx);

/* Free the context's device workspace (and its pinned staging) when larger
 * than keep_bytes; the next call allocates again.  Call only between calls on
 * the context (every entry point has finished its device work on return). */
int hpez_ctx_trim(hpez_ctx* ctx, uint64_t keep_bytes);

/* Cap the context's device workspace at max_workspace_bytes (0: no cap).  A
 * call that needs more fails with HPEZ_ENOMEM before any device work, and the
 * context stays usable: a server can bound each slot's memory and reject or
 * retry such requests. */
int hpez_ctx_set_limit(hpez_ctx* ctx, uint64_t max_workspace_bytes);

/* Current device workspace of the context in bytes (host-only). */
int hpez_ctx_workspace(const hpez_ctx* ctx, uint64_t* bytes);

/* Default configuration for a field: interpolation, linear 1D style in natural
 * order on every level, anchor stride by dimension count, R = 32768,
 * chunk = 1024, alpha = beta = 1, unit MD weights, no block-wise, no freeze. */
int hpez_config_default(const hpez_field_desc* desc, hpez_config* cfg);

/* Upper bound of the compressed size of any field matching desc/cfg.  Pure. */
int hpez_compress_bound(const hpez_field_desc* desc, const hpez_config* cfg, uint64_t* out_bytes);

/* Compress the device field d_in (desc) into the device buffer d_out of
 * out_cap bytes.  On success *out_size (host) is the stream length; the stream
 * is complete when the call returns.  Stream layout: a 512-byte header then
 * sections (block configs, anchors, verbatim values, Lorenzo outliers and
 * patches, code lengths, chunk bit counts, payload), little-endian, each on an
 * 8-byte boundary.  HPEZ_ENOSPC if out_cap is below the stream length. */
int hpez_compress(hpez_ctx* ctx, const hpez_field_desc* desc, const void* d_in,
                  const hpez_config* cfg, void* d_out, uint64_t out_cap, uint64_t* out_size,
                  hipStream_t stream);

/* Compress n fields in one call (many fields of uneven shapes and dtypes).
 * Arrays have n entries: desc[i], cfg[i] (host structs), d_in[i] and d_out[i]
 * (device pointers), out_cap[i]; out_sizes[i] (host) receives stream i's
 * length, 0 if field i failed.  Every field goes through the same steps as in
 * hpez_compress, so stream i is byte-identical to the plain call's; the batch
 * shares one stream synchronization per phase among all fields, runs the
 * per-block phase of all block-wise fields of a dtype in fused launches, and
 * builds the Huffman codebooks (Sec. 4 step 4) on several host threads.
 * Returns HPEZ_OK when every field succeeded, otherwise the error of the first
 * failing field (by dtype group, then index); a device error ends the call.
 * Device workspace is the sum of the fields' footprints. */
int hpez_compress_batch(hpez_ctx* ctx, int n, const hpez_field_desc* desc,
                        const void* const* d_in, const hpez_config* cfg, void* const* d_out,
                        const uint64_t* out_cap, uint64_t* out_sizes, hipStream_t stream);

/* Read the field description and size facts of a stream whose first bytes
 * (at least 512) are at h_hdr (host).  n_points / total_bytes may be NULL. */
int hpez_inspect(const void* h_hdr, uint64_t n, hpez_field_desc* desc, uint64_t* n_points,
                 uint64_t* total_bytes);

/* Decompress the device stream d_in (in_size bytes) into d_out (device,
 * out_cap bytes >= points * sizeof(dtype)).  HPEZ_ECORRUPT for a malformed
 * stream, HPEZ_ENOSPC if out_cap is too small.  Synchronises the stream to
 * read the header, then enqueues the rest. */
int hpez_decompress(hpez_ctx* ctx, const void* d_in, uint64_t in_size, void* d_out,
                    uint64_t out_cap, hipStream_t stream);

/* Decompress n streams in one call: d_in[i] (device, in_size[i] bytes) into
 * d_out[i] (device, out_cap[i] bytes).  rcs[i] (host) receives stream i's own
 * result (HPEZ_OK, HPEZ_ECORRUPT, HPEZ_ENOSPC).  Output i is bit-identical to
 * hpez_decompress of stream i; headers are read with one synchronization and
 * the per-block phase of all block-wise streams of a dtype runs in fused
 * launches.  Returns HPEZ_OK when every stream succeeded, otherwise the first
 * nonzero rcs[i]; a device error ends the call. */
int hpez_decompress_batch(hpez_ctx* ctx, int n, const void* const* d_in, const uint64_t* in_size,
                          void* const* d_out, const uint64_t* out_cap, int* rcs,
                          hipStream_t stream);

/* Decompression plans: the decompression of fixed streams into fixed outputs
 * (the inverse D_theta of Eq. 1, Sec. 4 steps 3-4 reversed) recorded once as
 * a HIP graph and replayed stream-ordered, with no host synchronisation and
 * no host work per replay.  For streams that are decompressed many times
 * (fields kept compressed in device memory and expanded on each read).
 *
 * hpez_decompress_plan takes the arguments of hpez_decompress_batch (device
 * streams d_in[i] of in_size[i] bytes, device outputs d_out[i] of out_cap[i]
 * bytes, rcs[i] per stream on the host) and runs that decompression once on
 * `stream` (synchronising it), which checks every stream and fills d_out;
 * any failure is returned as by hpez_decompress_batch and no plan is made.
 * It then records the same device work into a graph.  The plan holds its own
 * workspace and host staging (hpez_footprint's decompression need per
 * stream, plus the decode tables); `ctx` only lends its tuned launch shapes
 * (hpez_autotune), and may be used for other calls meanwhile.  d_in[i] and
 * d_out[i] are borrowed: they must stay allocated, and the streams' bytes
 * unchanged, while the plan lives.  Returns HPEZ_ENOMEM if the plan's memory
 * cannot be allocated, HPEZ_EDEVICE if recording or instantiation fails.
 *
 * hpez_plan_launch enqueues one replay on `stream` and returns; the outputs
 * are complete when the stream reaches that point and are bit-identical to
 * hpez_decompress_batch's.  Replays of one plan must not overlap (they share
 * the plan's workspace): keep them on one stream or order them with events.
 *
 * hpez_plan_status synchronises `stream` and reads the device status of the
 * last replay enqueued before it on that stream: rcs[i] (host, n entries)
 * receives HPEZ_OK or HPEZ_ECORRUPT for stream i, and the first nonzero one
 * is returned.
 *
 * hpez_plan_destroy waits for the last replay launched (an event recorded
 * after each launch), then frees the plan. */
typedef struct hpez_plan hpez_plan;
int hpez_decompress_plan(hpez_ctx* ctx, int n, const void* const* d_in, const uint64_t* in_size,
                         void* const* d_out, const uint64_t* out_cap, int* rcs,
                         hipStream_t stream, hpez_plan** out_plan);
int hpez_plan_launch(hpez_plan* plan, hipStream_t stream);
int hpez_plan_status(hpez_plan* plan, hipStream_t stream, int* rcs);
void hpez_plan_destroy(hpez_plan* plan);

/* Lossless stage after Huffman coding (Sec. 4, step 5), for any byte string
 * (normally a stream of hpez_compress).  The bytes become tokens: a nonzero
 * byte v is token v (1..255); a maximal run of k zero bytes is floor(k/4096)
 * tokens 4351 followed, when r = k mod 4096 is not 0, by token 255 + r.  The
 * tokens are Huffman-coded (canonical code, chunks of 1024, as the
 * quantization codes); if that is not smaller than the input, the input is
 * stored.  Container (little-endian): u32 magic "HPZL", u16 version 1, u16
 * mode (0 stored, 1 coded), u64 n, u64 n_tokens, u64 payload_bits, u32 chunk,
 * u32 sym_min, u32 sym_max, u32 run limit (4096); then the n bytes (mode 0),
 * or code lengths u8[sym_max - sym_min + 1], chunk bit counts
 * u16[ceil(n_tokens / 1024)] and payload u32[ceil(payload_bits / 32)], each
 * section starting 8-byte aligned (mode 1).
 *
 * hpez_lossless_bound: the largest container for n input bytes (48 + n).
 * hpez_lossless_encode: d_in (device, n bytes, n < 2^32 - 1, else
 *   HPEZ_EUNSUPPORTED) into d_out (device, out_cap >= the bound, else
 *   HPEZ_ENOSPC); *out_size (host) receives the container's size.
 *   Synchronises the stream (the codebook is built on the host).
 * hpez_lossless_decode: the container d_in (device, in_size bytes) into d_out
 *   (device, out_cap bytes); *out_size (host) receives n (also when out_cap is
 *   too small: HPEZ_ENOSPC).  HPEZ_ECORRUPT for a malformed container.  Reads
 *   the header with one synchronisation; a coded container synchronises again
 *   to check the decoding, a stored one returns after enqueueing its copy. */
int hpez_lossless_bound(uint64_t n, uint64_t* out_bytes);
int hpez_lossless_encode(hpez_ctx* ctx, const void* d_in, uint64_t n, void* d_out,
                         uint64_t out_cap, uint64_t* out_size, hipStream_t stream);
int hpez_lossless_decode(hpez_ctx* ctx, const void* d_in, uint64_t in_size, void* d_out,
                         uint64_t out_cap, uint64_t* out_size, hipStream_t stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): hpez_decompress on GPU
 * `device` with no allocation.  The device workspace is the library's static
 * 64 MiB per-GPU array (held by every GPU the library runs on until the
 * process ends); host staging is static too, and every kernel runs on
 * `stream` (no second stream).  d_in (in_size bytes) and d_out (out_cap
 * bytes) are caller device memory on `device`, as in hpez_decompress, whose
 * output this matches bit for bit.  A stream whose decompression needs more
 * workspace than the array fails with HPEZ_ENOMEM before any kernel runs
 * (hpez_footprint with op 1 gives the need; integer streams, which need a
 * float64 copy of the field, always fail so).  Calls on one GPU share its
 * array and its staging: they must not overlap (serialize them, e.g. on one
 * stream from one thread); the call clears what must start at zero.
 * Synchronises `stream` like hpez_decompress. */
int hpez_decompress_noalloc(int device, const void* d_in, uint64_t in_size, void* d_out,
                            uint64_t out_cap, hipStream_t stream);

/* Auto-tune a configuration for the device field d_in (Sec. 6).  *out_cfg is
 * in/out: on entry its radius, chunk, alpha and beta are used (the rest is
 * ignored); on return it holds a complete configuration.  When block-wise
 * tuning is on,
 * h_block_cfg (host, one byte per block, caller-owned, capacity
 * block_cfg_cap) receives the per-block choices and out_cfg->block_cfg points
 * to it.  Synchronous. */
int hpez_tune(hpez_ctx* ctx, const hpez_field_desc* desc, const void* d_in,
              const hpez_tune_opts* opts, hpez_config* out_cfg, uint8_t* h_block_cfg,
              uint64_t block_cfg_cap, hipStream_t stream);

/* Tune n fields in one call.  Arrays of n entries: desc[i], d_in[i] (device),
 * opts[i], out_cfg[i] (in/out as in hpez_tune), h_block_cfg[i] (host buffer of
 * block_cfg_cap[i] bytes, or NULL without block-wise tuning); rcs[i] receives
 * field i's own result.  Field i's configuration and block choices are the
 * same as hpez_tune's; the batch synchronizes once per tuning phase for all
 * fields and runs the candidate trials of every field (Sec. 6.2, 6.3, 6.6) in
 * fused launches.  Returns HPEZ_OK when every field succeeded, otherwise the
 * first nonzero rcs[i]; a device error ends the call.  Synchronous. */
int hpez_tune_batch(hpez_ctx* ctx, int n, const hpez_field_desc* desc, const void* const* d_in,
                    const hpez_tune_opts* opts, hpez_config* out_cfg, uint8_t* const* h_block_cfg,
                    const uint64_t* block_cfg_cap, int* rcs, hipStream_t stream);

/* Device bytes the context needs for op (0 compress, 1 decompress, 2 tune) of
 * such a field, beyond the caller's input and output buffers.  Pure. */
int hpez_footprint(const hpez_field_desc* desc, const hpez_config* cfg, int op, uint64_t* bytes);

/* Quality of a reconstruction xr of the field x: the functions M of the
 * requirement M(X, X') >= m0 in Sec. 3.1, Eq. (1).
 *   value_range  L = max(x) - min(x);
 *   max_abs_err  max |x - xr|;
 *   mse, psnr    mean (x - xr)^2 and 20 log10(L) - 10 log10(mse) (+inf when
 *                mse = 0, -inf when L = 0 < mse);
 *   ssim         mean over windows of the structural similarity
 *                ((2 mx my + C1)(2 sxy + C2)) / ((mx^2 + my^2 + C1)(sx^2 + sy^2 + C2)),
 *                C1 = (0.01 L)^2, C2 = (0.03 L)^2 (L taken as 1 when 0),
 *                population moments, uniform weights; windows are boxes of side
 *                w along every dim of size > 1 (a dim shorter than w is one
 *                window wide), without overlap from the origin; the partial
 *                windows at the far ends are left out (n_windows counts the
 *                others).
 * All sums are float64 in an order fixed by the sizes alone, so repeated
 * evaluations give the same bits. */
typedef struct {
  uint64_t n;
  uint64_t n_windows;
  double value_range;
  double max_abs_err;
  double mse;
  double psnr;
  double ssim;
} hpez_quality;

enum { HPEZ_METRIC_PSNR = 0, HPEZ_METRIC_SSIM = 1 };

/* Evaluate hpez_quality of d_xr against d_x (device arrays of desc's dtype and
 * dims; desc's bound fields are ignored).  ssim_window: window side w (0 = 8,
 * at most 64).  HPEZ_EINVAL for non-finite values.  Synchronous. */
int hpez_quality_eval(hpez_ctx* ctx, const hpez_field_desc* desc, const void* d_x, const void* d_xr,
                      uint32_t ssim_window, hpez_quality* out, hipStream_t stream);

/* Options of hpez_fit_eb.
 *   metric            HPEZ_METRIC_PSNR or HPEZ_METRIC_SSIM (target < 1);
 *   target            m0: the reconstruction must reach metric >= m0;
 *   steps_per_octave  G of the bound grid e_k = L 2^(k / G) (0 = 64);
 *   max_iter          compressions at most (0 = 12, at most 64);
 *   ssim_window       as in hpez_quality_eval (0 = 8). */
typedef struct {
  int32_t metric;
  uint32_t steps_per_octave;
  double target;
  uint32_t max_iter;
  uint32_t ssim_window;
} hpez_fit_opts;

/* Result of hpez_fit_eb: e (absolute bound, 0 when no tried bound met the
 * target), the quality and stream size of the compression at e, the number of
 * compressions run, and e_hi, the smallest tried bound that missed the target
 * (+inf when none did). */
typedef struct {
  double e;
  double e_hi;
  hpez_quality quality;
  uint64_t bytes;
  uint32_t iterations;
  uint32_t pad;
} hpez_fit_result;

/* The largest error bound on the grid e_k = L 2^(k / G) (L = value range of
 * the field) found whose compression of d_in under cfg meets the quality
 * requirement of Eq. (1), M(X, X') >= m0 (the compression ratio grows with
 * the bound, so this is the ratio-optimal bound for the requirement).  Search:
 * k starts at the model guess (PSNR: uniform errors on [-e, e], MSE = e^2 / 3;
 * SSIM: e = L / 1000); each step compresses and decompresses the whole field
 * at e_k on the device and measures the metric; met targets raise the floor
 * k_lo, missed ones lower the ceiling k_hi; the next k is the model step
 * (PSNR: 20 dB per decade of e; SSIM: deficit 1 - SSIM as e^2; at least one
 * step, at most four octaves) until both exist, then floor((k_lo + k_hi) / 2);
 * it ends when k_hi - k_lo <= 1 or after max_iter compressions.  desc's bound
 * fields are ignored (the compressions use absolute bounds); cfg as in
 * hpez_compress.  A constant field gives e = 0 (any bound reproduces it).
 * Allocates two device buffers for the trial stream and reconstruction.
 * Synchronous. */
int hpez_fit_eb(hpez_ctx* ctx, const hpez_field_desc* desc, const void* d_in,
                const hpez_config* cfg, const hpez_fit_opts* opts, hpez_fit_result* res,
                hipStream_t stream);

/* Launch shapes measured on the device (hpez_autotune).  A choice is cached in
 * the context per kernel kind (0: face steps, value = lanes per work-group |
 * points per lane << 16; 1: tuner region trials, value = lanes per work-group),
 * dtype class (0 float32, 1 float64 and integer fields) and size class (floor
 * log2 of the launch's points, resp. of a region's cells).  ms_before and
 * ms_best are the kind's kernel-group times under the previous shape and the
 * chosen one. */
typedef struct {
  int32_t kind;
  int32_t dtype;
  int32_t size_class;
  uint32_t value;
  double ms_before;
  double ms_best;
} hpez_tile_choice;

/* Measure launch shapes for the calls on this field and cache the fastest in
 * the context: the face steps of hpez_compress / hpez_decompress under cfg
 * (lanes per work-group 64, 128 or 256 times 1, 2, 4 or 8 points per lane),
 * and, when topts is not NULL, the region trials of hpez_tune (64, 256 or 1024
 * lanes).  Every size class the field's calls use is tried candidate by
 * candidate (best of three timed calls after a warm-up), the others keeping
 * their shapes.  Shapes never change a result.  Up to cap choices are written
 * to out; *n_out receives their number.  Allocates a stream and a
 * reconstruction buffer for the duration of the call.  Synchronous. */
int hpez_autotune(hpez_ctx* ctx, const hpez_field_desc* desc, const void* d_in,
                  const hpez_config* cfg, const hpez_tune_opts* topts, hpez_tile_choice* out,
                  int cap, int* n_out, hipStream_t stream);

/* Per-kernel timing (tracing aid).  While enabled, every kernel group the
 * context launches is bracketed by HIP events on its stream; each entry point
 * folds the elapsed times into per-name totals before returning.  `bytes` is
 * the algorithmic HBM traffic of the group (what the method must move: inputs
 * read once, outputs written once), so bytes / time is the achieved rate
 * against the HBM roofline.  Enabling clears the totals. */
typedef struct {
  char name[32];
  uint64_t launches;
  uint64_t bytes;
  double total_ms;
} hpez_kernel_stat;

int hpez_profile_enable(hpez_ctx* ctx, int on);
/* While profiling: record only the spans of the group named `group` (one of
 * the names hpez_profile_read reports), so that timing one group costs two
 * events per launch instead of two per group; NULL or "" records all groups
 * again.  The setting stays until changed. */
int hpez_profile_only(hpez_ctx* ctx, const char* group);
/* Copy up to cap entries into out; *n receives the number of entries. */
int hpez_profile_read(hpez_ctx* ctx, hpez_kernel_stat* out, int cap, int* n);

#ifdef __cplusplus
}
#endif

#endif /* HPEZ_H */
