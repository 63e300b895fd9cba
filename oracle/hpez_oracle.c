/*
 * hpez_oracle.c -- plain CPU oracle for the HPEZ compression hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is loaded by the test suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark; the product
 * library never links, loads or calls it, and the two share no source,
 * header, table or helper.
 *
 * What it computes (Liu et al., "High-performance Effective Scientific
 * Error-bounded Lossy Compression with Auto-tuned Multi-component
 * Interpolation"):
 *   - the compression pipeline of Sec. 4 (steps 2-4): level-wise anchor based
 *     interpolation prediction (Sec. 5.1), linear-scale quantization of the
 *     prediction error with the reconstructed value written back for later
 *     predictions (step 3 of Sec. 4), Huffman coding of the codes (step 4);
 *   - the spline stencils of Eq. (2), (6), (8), (13), (14);
 *   - multi-dimensional interpolation, Eq. (9) with weights from Eq. (12);
 *   - same-level cubic re-ordering (Sec. 5.4.2);
 *   - dimension freezing (Sec. 6.3) and block-wise configurations (Sec. 6.6);
 *   - level-wise error bounds, Eq. (15);
 *   - the value-range-relative error bound e = eps * (max - min) (Sec. 7.1.3);
 *   - a first-order Lorenzo predictor as the alternative of Sec. 6.5;
 *   - the auto-tuner of Sec. 6 (sampling statistics, global tuning, freezing,
 *     Lorenzo selection, block-wise tuning).
 * Where the paper leaves a detail open, the reading taken is stated at the
 * place it is used.
 *
 * Style: single-threaded scalar code, one point at a time, in the order the
 * method defines.  All floating-point expressions are written out in the order
 * they are evaluated; the file must be compiled with -ffp-contract=off and
 * without -ffast-math.
 *
 * Parity status of each function is stated in its comment.  Anything computed
 * from the paper's printed numbers is pinned by the tests under tests/.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_ECORRUPT -4
#define ORC_ENOSPC -5
#define ORC_EUNSUPPORTED -6
#define ORC_ESCHEDULE -7 /* internal: a stencil read a point not yet known */

#define ORC_LIN 0
#define ORC_NAK 1
#define ORC_NAT 2

/* One interpolation configuration: a level's (or a block's) choice among the
 * options tuned in Sec. 6.2. */
typedef struct {
  uint8_t kind;       /* 0 linear Eq.(2), 1 not-a-knot cubic Eq.(6), 2 natural cubic Eq.(8) */
  uint8_t md;         /* 0 one dimension at a time, 1 multi-dimensional Eq.(9) */
  uint8_t same_level; /* cubic + 1D style only: Sec. 5.4.2 two-step split */
  uint8_t order[4];   /* 1D style: dimension index of each pass, first pass first */
  uint8_t pad;
} orc_interp;

/* Everything the compressor needs besides the data. */
typedef struct {
  uint8_t dtype;       /* 0 float32, 1 float64; integers 2 uint8, 3 uint16, 4 int16, 5 int32:
                          the method runs in double on their values (the caller passes
                          doubles) with reconstructions rounded to integers */
  uint8_t ndims;       /* 1..4 */
  uint8_t eb_mode;     /* 0 absolute, 1 value-range relative */
  uint8_t predictor;   /* 0 interpolation, 1 Lorenzo */
  uint8_t anchor_log2; /* anchor stride A = 2^anchor_log2 */
  uint8_t block_log2;  /* 0: no block-wise configs; else block side B = 2^block_log2 */
  int8_t frozen_dim;   /* -1: none */
  uint8_t pad0;
  uint32_t radius;     /* quantization radius R; codes are q + R, 0 = unpredictable */
  uint32_t chunk;      /* Huffman chunk length in symbols */
  uint64_t dims[4];    /* row-major, last index fastest */
  double eb;           /* user error bound (absolute, or relative to the value range) */
  double alpha, beta;  /* Eq. (15) */
  double md_w[3][4];   /* per stencil kind, per dim: the 1/sigma^2 weight of Eq. (12) */
  orc_interp level[16];/* level l (stride 2^(l-1)) uses level[l-1] */
  orc_interp cand[16]; /* block-wise candidates */
  uint32_t n_cand;
  uint32_t pad1;
  const uint8_t* block_cfg; /* one candidate index per block (row-major blocks) */
} orc_params;

/* ------------------------------------------------------------------ */
/* geometry                                                            */
/* ------------------------------------------------------------------ */

typedef struct {
  int D;            /* always 4: trailing dims padded with size 1 */
  int64_t n[4];
  int64_t st[4];    /* row-major strides */
  int64_t N;
  int act[4];       /* dim takes part in interpolation (size > 1 and not frozen) */
  int nact;
} geom;

static void geom_init(geom* g, const uint64_t* dims, int ndims, int frozen)
{
  g->D = 4;
  for (int d = 0; d < 4; d++) g->n[d] = d < ndims ? (int64_t)dims[d] : 1;
  g->st[3] = 1;
  for (int d = 2; d >= 0; d--) g->st[d] = g->st[d + 1] * g->n[d + 1];
  g->N = g->st[0] * g->n[0];
  g->nact = 0;
  for (int d = 0; d < 4; d++) {
    g->act[d] = (g->n[d] > 1 && d != frozen);
    g->nact += g->act[d];
  }
}

/* ------------------------------------------------------------------ */
/* error bounds: Sec. 7.1.3 (value-range relative) and Eq. (15)         */
/* ------------------------------------------------------------------ */

/* Level error bound of Eq. (15): e_l = e / min(alpha^(l-1), beta).  The power is
 * formed by repeated multiplication from the left.  Level 1 (the finest) always
 * gets e itself, as Sec. 5.1 requires of the last level. */
static double level_eb(double e, double alpha, double beta, int l)
{
  double pw = 1.0;
  for (int i = 1; i < l; i++) pw = pw * alpha;
  double m = pw < beta ? pw : beta;
  if (l == 1) m = 1.0;
  return e / m;
}

/* ------------------------------------------------------------------ */
/* quantizer (Sec. 4, step 3)                                          */
/* ------------------------------------------------------------------ */
/* The paper fixes only |e_q - e| <= eps.  Reading taken: bins of width 2*e_l,
 * round half away from zero, radius R, arithmetic in double, and a post-check
 * that sends a point to the verbatim list when the value the decompressor
 * will rebuild misses the bound (or any quantity is not finite). */
/* Integer fields (rnd): the rebuilt value is rounded to the nearest integer
 * (ties to even) before the check, so the working grid holds integers. */
#define QUANT_BODY(T)                                                          \
  double t = ((double)x - (double)p) * inv2e;                                  \
  double qf = floor(fabs(t) + 0.5);                                            \
  if (!(qf < (double)R)) return 0;                                             \
  double q = t < 0 ? -qf : qf;                                                 \
  double v = (double)p + q * twoe;                                             \
  T xr = (T)(rnd ? rint(v) : v);                                               \
  if (!(fabs((double)xr - (double)x) <= el)) return 0;                         \
  *xr_out = xr;                                                                \
  return (uint16_t)((int64_t)q + (int64_t)R);

static uint16_t quantize_f(float x, float p, double inv2e, double twoe, double el, uint32_t R,
                           int rnd, float* xr_out) { QUANT_BODY(float) }
static uint16_t quantize_d(double x, double p, double inv2e, double twoe, double el, uint32_t R,
                           int rnd, double* xr_out) { QUANT_BODY(double) }

/* ------------------------------------------------------------------ */
/* type-generic core: instantiated for float and double                */
/* ------------------------------------------------------------------ */

#define T float
#define SFX(name) name##_f
#define QUANTIZE quantize_f
#define K6 0x1.555556p-3f
#define K40 0x1.99999ap-6f
#define K62 0x1.084210p-6f
#include "oracle_core.inc"
#undef T
#undef SFX
#undef QUANTIZE
#undef K6
#undef K40
#undef K62

#define T double
#define SFX(name) name##_d
#define QUANTIZE quantize_d
#define K6 0x1.5555555555555p-3
#define K40 0x1.999999999999ap-6
#define K62 0x1.0842108421084p-6
#include "oracle_core.inc"
#undef T
#undef SFX
#undef QUANTIZE
#undef K6
#undef K40
#undef K62

#include "oracle_huffman.inc"
#include "oracle_stream.inc"
#include "oracle_tune.inc"
