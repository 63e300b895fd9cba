// tune_dev.h -- shared declarations of the auto-tuner kernels (Sec. 6).
#pragma once

#include "hpez_internal.h"

namespace hpez {

constexpr size_t kTrialLdsBytes = 48 * 1024;  // regions up to this size run from LDS
constexpr uint32_t kTrialHistWin = 4096;      // histogram bins kept in LDS (codes hist_lo ...)
constexpr size_t kTrialBoxLdsBytes = 160 * 1024 - 256;  // in-LDS regions of up to three dims

// A trial region: origin and extents inside the field.
struct TrialBox {
  int64_t o[4];
  int64_t m[4];
};

struct TrialArgs {
  Geom fg;             // field geometry (for addressing X)
  int32_t frozen;      // frozen dim of the trial, -1 none
  int32_t L;           // anchor_log2 of the region
  uint32_t R;
  int32_t tuned;       // 1: level[] per level; 0: candidate blockIdx.y on every level
  int32_t score_mode;  // 0: score[cand][level] summed over regions; 1: score[region][cand];
                       // 2: score[0] += the distortion of Sec. 6.4 (sum of
                       //    floor(((x - x') * inv_e)^2 * 2^32) over predicted points)
  uint32_t hist_lo;    // first code of the LDS histogram window
  int32_t max_ext;     // largest region extent along any dim
  int32_t pad2;
  uint64_t box_cap;    // points of the largest region (scratch stride)
  double score_mul;    // 4096 / e
  double inv_e;        // 1 / e (score_mode 2)
  double el[17], inv2e[17], twoe[17];
  hpez_interp cand[16];
  hpez_interp level[16];
  double wmd[3 * 8 * 4];  // MD weights [kind][odd set][dim] (Eq. 12), first three dims
};

// One tuning run's trials in a fused launch: n_boxes regions x n_cand
// candidates, work-groups [wg_begin, wg_begin + n_boxes * n_cand) of the launch.
template <typename T>
struct TrialJob {
  TrialArgs a;
  const TrialBox* boxes;
  const T* X;
  unsigned long long* score;
  uint32_t* hist;
  uint32_t n_boxes, n_cand;
  uint64_t wg_begin;
};

#ifdef __HIPCC__
// Sum over the work-group; every thread receives the total.
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v,
                                                            unsigned long long* red)
{
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  unsigned long long t = 0;
  const int nw = (blockDim.x + 63) / 64;
  for (int w = 0; w < nw; w++) t += red[w];
  return t;
}
#endif

// d_sums: kStatSlots copies of the 12 sums (zeroed); work-group w adds into
// copy w % kStatSlots, so the atomics of many work-groups do not all meet on
// the same 12 words.  The caller adds the copies (integers: exact in any order).
constexpr int kStatSlots = 64;
template <typename T>
hipError_t launch_stats(const T* X, const Geom& g, const Lattice& lat, double mul,
                        unsigned long long* d_sums, hipStream_t st);
template <typename T>
hipError_t launch_trials(const TrialArgs& a, const TrialBox* d_boxes, uint32_t n_boxes,
                         uint32_t n_cand, const T* X, T* scratch, const double* d_wq,
                         unsigned long long* d_score, uint32_t* d_hist, hipStream_t st);
// regions that fit the in-LDS box kernel (the fused launches take only these)
template <typename T>
bool trial_box_ok(const TrialArgs& a, bool hist);
template <typename T>
size_t trial_box_lds(const TrialArgs& a, bool hist);
// entries [0, n) of d_jobs in one launch of total_wg work-groups of `lanes`
// threads (64, 256 or 1024, by region size); lds = the largest entry's
// trial_box_lds
template <typename T>
hipError_t launch_trial_jobs(const TrialJob<T>* d_jobs, const uint64_t* d_wg_begin, int n,
                             uint64_t total_wg, size_t lds, bool hist, int lanes, hipStream_t st);
// lanes per trial work-group for a region of box_cap points
inline int trial_lanes(uint64_t box_cap) { return box_cap > 4096 ? 1024 : box_cap > 1536 ? 256 : 64; }
template <typename T>
hipError_t launch_lorenzo_trial(const Geom& fg, const TrialBox* d_boxes, uint32_t n_boxes,
                                uint32_t max_pts, const T* X, double inv2e, uint32_t R,
                                uint32_t hist_lo, uint32_t* d_hist, int* d_unsupported,
                                hipStream_t st);
// The nonzero bins of a histogram as (bin, count) pairs, in no particular
// order, for the host's entropy estimate: *d_count (zeroed by the caller)
// receives their number; pairs beyond cap are dropped (the caller then reads
// the whole histogram).
constexpr uint32_t kNzCap = 2048;
hipError_t launch_hist_nonzero(const uint32_t* d_hist, uint32_t nsym, uint32_t* d_count,
                               uint32_t* d_pairs, uint32_t cap, hipStream_t st);
// the same for n histograms stored back to back (nsym bins each): counts
// d_count[0, n), pairs of histogram i at d_pairs + 2 cap i
hipError_t launch_hist_nonzero_set(const uint32_t* d_hist, uint32_t nsym, uint32_t n,
                                   uint32_t* d_count, uint32_t* d_pairs, uint32_t cap,
                                   hipStream_t st);
// first code of a kTrialHistWin-wide window centred on R inside [0, 2R)
inline uint32_t trial_hist_lo(uint32_t R)
{
  const uint32_t nsym = 2 * R;
  uint32_t lo = R > kTrialHistWin / 2 ? R - kTrialHistWin / 2 : 0;
  if (lo + kTrialHistWin > nsym) lo = nsym > kTrialHistWin ? nsym - kTrialHistWin : 0;
  return lo;
}

}  // namespace hpez
