// lorenzo_dev.h -- declarations of the Lorenzo alternative's kernels (Sec. 6.5).
#pragma once

#include "hpez_internal.h"

namespace hpez {

struct LorenzoArgs {
  double inv2e;   // 1 / (2e)
  double twoe;    // 2e
  double e;       // bound checked after reconstruction
  uint32_t R;
  uint32_t chunk;
};

template <typename T>
hipError_t launch_lorenzo_codes(const T* X, const Geom& g, uint64_t n, const LorenzoArgs& a,
                                uint16_t* code, uint32_t* pcount, int* bad, hipStream_t st);
template <typename T>
hipError_t launch_lorenzo_gather(const T* X, const Geom& g, uint64_t n, const LorenzoArgs& a,
                                 const uint16_t* code, const uint32_t* czero, const uint64_t* zoff,
                                 const uint32_t* pcount, const uint64_t* poff, long long* outl,
                                 uint64_t* pidx, T* pval, hipStream_t st);
template <typename T>
hipError_t launch_lorenzo_rebuild(const uint16_t* code, const Geom& g, uint64_t n, uint32_t R,
                                  uint32_t chunk, const uint32_t* czero, const uint64_t* zoff,
                                  const long long* outl, uint64_t n_outl, const uint64_t* pidx,
                                  const T* pval, uint64_t n_patch, double twoe, long long* v,
                                  T* out, int* status, hipStream_t st);

}  // namespace hpez
