// hpez_internal.h -- shared declarations of the HIP kernels and the host
// runtime of the MI355X HPEZ library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hpez.h"

namespace hpez {

constexpr int kMaxLevels = 16;
constexpr int kHdrBytes = 512;
constexpr uint32_t kMagic = 0x5A455048u;  // "HPEZ"
constexpr int kLmax = 32;                 // longest Huffman codeword
constexpr int kLutBits = 12;              // first-level decode table width
constexpr int kBrickLog2 = 5;             // code order: bricks of 32 points per dim

// Grid geometry, always padded to four dims (size-1 dims are inactive).
struct Geom {
  int64_t n[4];
  int64_t st[4];
  int32_t act[4];
};

// A lattice {first_d + k * step_d, k < cnt_d} in every dim.
struct Lattice {
  int64_t first[4];
  int64_t step[4];
  uint32_t cnt[4];
  uint64_t total;
};

// One step (pass, half pass or multi-dimensional sub-step) of one level.
struct StepArgs {
  Geom g;
  Lattice lat;
  int64_t s;          // stride of the level
  int64_t B;          // block side (face filter), 0 = none
  int32_t filter;     // 0 all lattice points, 1 only points on block faces
  int32_t kind;       // 0 linear, 1 not-a-knot, 2 natural
  int32_t md;         // multi-dimensional
  int32_t sl;         // same-level second half
  int32_t pdim;       // pass dimension (1D style)
  uint32_t odd;       // odd set (multi-dimensional)
  double wq[4];       // normalised MD weights for this odd set (double, cast to T on use)
  double el, inv2e, twoe;
  uint32_t R;
  int32_t mdhalf;     // multi-dimensional same-level: 0 all points, 1 + c only colour c
  // block faces (filter): the lattice points whose coordinate along face
  // dim fdim[f] is a multiple of B, f < nface, filled in by the launcher
  int32_t nface;
  int32_t fdim[4];
  Lattice flat[4];
  uint64_t fstart[5];
};

// Interior points of every block at one level, one step index of each block's
// own configuration.
struct BlockStepArgs {
  Geom g;
  Lattice lat;        // the level's coarse lattice (multiples of s on active dims)
  int64_t s, B;
  int64_t nb[4];
  int32_t t;          // step index processed by this launch
  uint32_t pieces;    // work-groups per block
  double el, inv2e, twoe;
  uint32_t R;
  hpez_interp cand[16];
};

// Launchers (defined in the .hip files).  All return hipError_t.
template <typename T>
hipError_t launch_step(const StepArgs& a, const T* X, T* W, uint16_t* code, int mode,
                       hipStream_t st);
template <typename T>
hipError_t launch_block_step(const BlockStepArgs& a, const T* X, T* W, uint16_t* code,
                             const uint8_t* d_block_cfg, const double* d_wq, int mode,
                             hipStream_t st);
template <typename T>
hipError_t launch_anchors(const Geom& g, const Lattice& lat, const T* X, T* W, uint16_t* code,
                          T* out_anchor, uint32_t R, int mode, hipStream_t st);
template <typename T>
hipError_t launch_minmax(const T* X, uint64_t n, double* d_part, int* d_bad, int nblocks,
                         hipStream_t st);
hipError_t launch_minmax_final(double* d_part, int nblocks, double* d_out, hipStream_t st);

// Huffman
hipError_t launch_histogram(const uint16_t* code, uint64_t n, uint32_t* hist, uint32_t nsym,
                            uint32_t R, hipStream_t st);
hipError_t launch_scan_u32_to_u64(const uint32_t* in, uint64_t n, uint64_t* out_excl,
                                  uint64_t* d_total, uint64_t* tmp, hipStream_t st);
hipError_t launch_u16_to_u32(const uint16_t* in, uint64_t n, uint32_t* out, hipStream_t st);

}  // namespace hpez
