// block_dev.h -- declarations of the block-wise kernels (k_block.hip).
#pragma once

#include "hpez_internal.h"

namespace hpez {

constexpr int kBlockHistWin = 4096;  // LDS histogram window of the block kernel
constexpr int kBlockThreads = 1024;  // work-group size of the block kernel
constexpr int kSmallBoxThreads = 256;  // ... for boxes of at most two active dims
// coarse levels on the block lattice: levels above kCoarseL (strides >= 4);
// a block's lattice has at most 9 x 9 x 32 cells (one inactive dim of 32)
constexpr int kCoarseL = 2;
constexpr int kCoarseCells = 9 * 9 * 32;

// Compact face arrays: family e holds the planes x_e = 0, B, 2B, ... with layout
// [plane][other dims row-major]; index = (x_e / B) * plane[e] + sum_k x_k fs[e][k].
struct FaceGeo {
  void* val[4];        // T values per family (nullptr for inactive dims)
  uint16_t* code[4];   // compress: codes of the points whose lowest face family is d
  int64_t plane[4];    // points per plane
  int64_t fs[4][4];    // strides of the other dims inside a plane (fs[e][e] = 0)
  int64_t B;
  int32_t blog2;
  int32_t pad;
};

// One step of the face phase over every family it touches.  The step's
// lattice (first/step/cnt per dim) is shared; family d enumerates its planes
// x_d = 0, B, 2B, ... (slowest) times the lattice of the other dims, and owns
// the launch indices [off[d], off[d + 1]).
struct FaceStep {
  Geom g;
  int64_t first[4], step[4];
  uint32_t cnt[4];
  uint32_t mg[4];   // magic multipliers for division by cnt (32-bit indices)
  int32_t msh[4];   // their shifts (-1: cnt <= 1)
  uint64_t off[5];
  int32_t kind, md, sl, pdim;
  uint32_t odd;
  uint32_t R;
  double wq[4];
  int64_t s;
  double el, inv2e, twoe;
  int32_t mdhalf;  // multi-dimensional same-level: 0 all points, 1 + c only colour c
  int32_t pad;
};

struct BlockArgs {
  Geom g;
  int64_t nb[4];       // blocks per dim (block side 32)
  int32_t L;           // levels handled: stride 2^(L-1) .. 1
  uint32_t R;
  uint32_t hist_lo;    // first symbol of the LDS histogram window
  int32_t vec;         // rows along dim 2 are 16-byte aligned in X / out / face arrays
  double el_l[17], inv2e_l[17], twoe_l[17];
  double wmd[3 * 8 * 4];  // MD weights [kind][odd set][dim] (Eq. 12), first three dims
  hpez_interp cand[16];
};

// Work tables of the fused launches (many fields in one launch).  A face-step
// entry owns work-groups [wg_begin, wg_begin + wg_count) of its launch; a block
// job owns global block indices [block_begin, block_begin + nb0 nb1 nb2).
template <typename T>
struct FaceEntry {
  FaceStep a;
  FaceGeo f;
  const T* X;
  uint16_t* code;
  const T* out;
  uint64_t wg_begin, wg_count;
  int32_t xface;   // compress: family 2's face array holds the original values (minmax_faces)
  int32_t fcode2;  // decompress: f.code[2] holds the codes of family 2 (the decoder's copy)
};

template <typename T>
struct BlockJobDev {
  BlockArgs a;
  FaceGeo f;
  const T* X;
  uint16_t* code;
  const uint8_t* bcfg;
  uint32_t* hist;
  T* out;
  T* cval;          // per block kCoarseCells lattice values (coarse levels' output)
  uint16_t* ccode;  // per block kCoarseCells lattice codes (compress)
  uint64_t block_begin;
};

// The coarse face levels (s >= 4) of one family of one field: one work-group
// per plane x_d = B p, the plane's lattice (every 4th point along its active
// dims) in LDS.  Work-groups [wg_begin, wg_begin + planes) of the launch.
template <typename T>
struct PlaneJob {
  Geom g;
  FaceGeo f;
  const T* X;
  const uint16_t* code;  // decompress: the codes (stream order)
  const T* out;          // decompress: the field (verbatim values)
  int32_t d;             // family: the planes' normal dim
  int32_t Ltop;          // first level (log2 B)
  int32_t E[3];          // lattice extents (1 along d)
  uint32_t mg_b0, mg_e2;  // magic multipliers / shifts for cell index / (E1 E2) and / E2
  int32_t sh_b0, sh_e2;
  uint32_t R;
  double el_l[17], inv2e_l[17], twoe_l[17];
  double wmd[3 * 8 * 4];
  hpez_interp level[16];  // the global configuration per level
  uint64_t wg_begin;
};

template <typename T>
hipError_t launch_planes(const PlaneJob<T>* d_tab, const uint64_t* d_wg_begin, int n,
                         uint64_t total_wg, size_t lds, int mode, hipStream_t st);

// one fused face step: entries [0, n) of the device table, total work-groups
template <typename T>
hipError_t launch_face_steps(const FaceEntry<T>* d_tab, const uint64_t* d_wg_begin, int n,
                             uint64_t total_wg, bool narrow, int mode, uint32_t threads,
                             hipStream_t st);
// the block phase of jobs [0, n): d_begin[j] = first global block index of job j
// (d_begin[n] = total); lds = largest box of the jobs; small: every job's box
// has at most two active dims (the 256-lane kernel, four work-groups per CU)
template <typename T>
hipError_t launch_block_jobs(const BlockJobDev<T>* d_jobs, const uint64_t* d_begin, int n,
                             uint64_t total_blocks, size_t lds, int n_cu, int mode, bool small,
                             hipStream_t st);

// the coarse levels of every block of jobs [0, n) on the block lattices
template <typename T>
hipError_t launch_coarse_jobs(const BlockJobDev<T>* d_jobs, const uint64_t* d_begin, int n,
                              uint64_t total_blocks, int mode, hipStream_t st);
// Value range (per-block partials and the non-finite flag, as launch_minmax)
// and, in the same pass over the field, the original values of the points of
// the face planes normal to dim 2 into that family's face array.  Up to three
// dims (n[3] == 1), rows along dim 2, fewer than 2^32 rows.
template <typename T>
hipError_t launch_minmax_faces(const T* X, const Geom& g, const FaceGeo& f, double* part, int* bad,
                               int nblocks, hipStream_t st);
template <typename T>
hipError_t launch_face_init(const FaceGeo& f, const Geom& g, const Lattice& lat, const T* W,
                            const uint16_t* code, int mode, hipStream_t st);
template <typename T>
size_t block_lds_bytes(const Geom& g);
}  // namespace hpez
