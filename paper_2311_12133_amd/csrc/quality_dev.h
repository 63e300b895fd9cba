// quality_dev.h -- declarations of the quality reductions (Sec. 3.1, Eq. 1).
#pragma once

#include "hpez_internal.h"

namespace hpez {

// SSIM windows of a field (4 dims, row-major, last fastest): side s[d] and
// count nw[d] per dim, element strides st[d] (st[3] = 1); cells = prod s[d];
// c1 = (0.01 L)^2 and c2 = (0.03 L)^2 with L the value range.
struct SsimGeom {
  int64_t s[4];
  uint64_t nw[4];
  int64_t st[4];
  uint64_t windows;
  uint32_t cells;
  uint32_t pad;
  double c1, c2;
};

// reduction layout: parts work-groups of per consecutive items each
struct QGrid {
  uint64_t per;
  uint32_t parts;
};
constexpr uint32_t kQMaxParts = 4096;
QGrid quality_grid(uint64_t n);

// d_part: 4 kQMaxParts doubles; d_out (4 doubles): sum of squared errors,
// max |error|, min x, max x
template <typename T>
hipError_t launch_quality_sums(const T* x, const T* xr, uint64_t n, double* d_part, double* d_out,
                               hipStream_t st);
// d_win: g.windows doubles (per-window SSIM); d_part: kQMaxParts doubles;
// d_out: the sum of the windows' SSIM
template <typename T>
hipError_t launch_ssim(const T* x, const T* xr, const SsimGeom& g, double* d_win, double* d_part,
                       double* d_out, hipStream_t st);

}  // namespace hpez
