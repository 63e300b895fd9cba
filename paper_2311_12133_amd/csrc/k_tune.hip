// k_tune.hip -- auto-tuner kernels (Sec. 6), gfx950.
//
//  * stats_kernel: the sampling statistics of Sec. 6.1 -- open-loop 1D linear,
//    not-a-knot and natural prediction errors along every dimension on a
//    sparse lattice, accumulated as integer sums of squared fixed-point errors.
//  * trial_kernel: closed-loop trial compressions of Sec. 6.2/6.3/6.6.  One
//    work-group per (region, candidate) runs the whole level schedule of the
//    region treated as a small field (its own anchors), predicting,
//    quantizing and writing reconstructions exactly as compression does, and
//    sums the integer error score per level (or per region); optionally it
//    histograms the codes for the size estimate.  Steps are separated by
//    work-group barriers; the region's working grid lives in LDS when it fits.
//  * lorenzo_trial_kernel: codes of the first-order Lorenzo predictor on the
//    same regions (Sec. 6.5), histogrammed.
// All scores are integers, so decisions are independent of summation order.

#include "box_dev.h"
#include "interp_dev.h"
#include "tune_dev.h"

namespace hpez {

// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) stats_kernel(const T* __restrict__ X, Geom g, Lattice lat,
                                                    double mul, unsigned long long* __restrict__ sums)
{
  unsigned long long acc[3][4];
  for (int k = 0; k < 3; k++)
    for (int d = 0; d < 4; d++) acc[k][d] = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < lat.total; k += stride) {
    int64_t x[4];
    lattice_point(lat, k, x);
    const int64_t idx = x[0] * g.st[0] + x[1] * g.st[1] + x[2] * g.st[2] + x[3];
    const T xv = X[idx];
    for (int d = 0; d < 4; d++) {
      if (!g.act[d]) continue;
      const int64_t sd = g.st[d];
      const T a = X[idx - 3 * sd], b = X[idx - sd], c = X[idx + sd], dd = X[idx + 3 * sd];
      T p[3];
      p[0] = (b + c) * (T)0.5;
      p[1] = ((b + c) * (T)9 - (a + dd)) * (T)0.0625;
      p[2] = ((b + c) * (T)23 - (a + dd) * (T)3) * SplineK<T>::k40();
      for (int kk = 0; kk < 3; kk++) {
        const double t = fabs((double)xv - (double)p[kk]) * mul;
        const unsigned long long q = (t < 1048576.0) ? (unsigned long long)floor(t) : 1048576ull;
        acc[kk][d] += q * q;
      }
    }
  }
  __shared__ unsigned long long red[256];
  for (int k = 0; k < 3; k++)
    for (int d = 0; d < 4; d++) {
      if (!g.act[d]) continue;
      const unsigned long long v = block_sum_u64(acc[k][d], red);
      if (threadIdx.x == 0 && v) atomicAdd(&sums[(blockIdx.x % kStatSlots) * 12 + k * 4 + d], v);
    }
}

template <typename T>
hipError_t launch_stats(const T* X, const Geom& g, const Lattice& lat, double mul,
                        unsigned long long* d_sums, hipStream_t st)
{
  if (lat.total == 0) return hipSuccess;
  uint64_t b = (lat.total + 255) / 256;
  if (b > 2048) b = 2048;
  hipLaunchKernelGGL((stats_kernel<T>), dim3((unsigned)b), dim3(256), 0, st, X, g, lat, mul, d_sums);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// one step of a trial over a region-local lattice
template <typename T, typename P>
__device__ void trial_step(const TrialArgs& a, const TrialBox& bx, const int64_t* bst,
                           const T* __restrict__ X, P* W, const int64_t* r, const int64_t* m,
                           int kind, int md, int sl, int pd, unsigned odd, int64_t s, int level,
                           const double* __restrict__ wq, unsigned long long& score,
                           uint32_t* __restrict__ hist, uint32_t* lh, unsigned long long& sq)
{
  uint32_t cnt[4];
  uint64_t total = 1;
  for (int d = 0; d < 4; d++) {
    cnt[d] = r[d] <= bx.m[d] - 1 ? (uint32_t)((bx.m[d] - 1 - r[d]) / m[d] + 1) : 0;
    total *= cnt[d];
  }
  const double el = a.el[level], inv2e = a.inv2e[level], twoe = a.twoe[level];
  const bool narrow = total <= 0xffffffffull;
  for (uint64_t k = threadIdx.x; k < total; k += blockDim.x) {
    int64_t x[4];
    if (narrow) {
      uint32_t rr = (uint32_t)k;
      for (int d = 3; d >= 0; d--) {
        const uint32_t q = rr / cnt[d];
        x[d] = r[d] + (int64_t)(rr - q * cnt[d]) * m[d];
        rr = q;
      }
    } else {
      uint64_t rr = k;
      for (int d = 3; d >= 0; d--) {
        const uint64_t q = rr / cnt[d];
        x[d] = r[d] + (int64_t)(rr - q * cnt[d]) * m[d];
        rr = q;
      }
    }
    const int64_t idx = x[0] * bst[0] + x[1] * bst[1] + x[2] * bst[2] + x[3];
    const int64_t fidx = (bx.o[0] + x[0]) * a.fg.st[0] + (bx.o[1] + x[1]) * a.fg.st[1] +
                         (bx.o[2] + x[2]) * a.fg.st[2] + (bx.o[3] + x[3]);
    T p;
    if (!md) {
      p = spline<T, P>(W, idx, s * pick4(bst, pd), pick4(x, pd), s, 0, pick4(bx.m, pd) - 1, kind,
                       sl);
    } else {
      bool first = true;
      T acc = (T)0;
      for (int d = 0; d < 4; d++) {
        if (!(odd >> d & 1u)) continue;
        const T pv = spline<T, P>(W, idx, s * bst[d], x[d], s, 0, bx.m[d] - 1, kind, 0);
        const T term = (T)wq[(kind * 16 + odd) * 4 + d] * pv;
        acc = first ? term : acc + term;
        first = false;
      }
      p = acc;
    }
    const T xv = X[fidx];
    const double t = fabs((double)xv - (double)p) * a.score_mul;
    score += (t < 4294967296.0) ? (unsigned long long)floor(t) : 4294967296ull;
    T xr = xv;
    const uint32_t q = quantize<T>(xv, p, inv2e, twoe, el, a.R, xr);
    W[idx] = q ? xr : xv;
    if (a.score_mode == 2) {
      const double u = ((double)xv - (double)xr) * a.inv_e;
      sq += (unsigned long long)floor(u * u * 4294967296.0);
    }
    if (hist) hist_add_wave(lh, hist, a.hist_lo, kTrialHistWin, q, true);
  }
}

template <typename T, typename P>
__device__ void trial_body(const TrialArgs& a, const TrialBox& bx, const T* __restrict__ X, P* W,
                           int cand, const double* __restrict__ wq,
                           unsigned long long* __restrict__ score, uint32_t* __restrict__ hist,
                           uint32_t* lh)
{
  __shared__ unsigned long long red[256];
  if (hist)
    for (uint32_t i = threadIdx.x; i < kTrialHistWin; i += blockDim.x) lh[i] = 0;
  int32_t act[4];
  int64_t bst[4];
  bst[3] = 1;
  for (int d = 2; d >= 0; d--) bst[d] = bst[d + 1] * bx.m[d + 1];
  int nact = 0;
  for (int d = 0; d < 4; d++) {
    act[d] = (bx.m[d] > 1 && d != a.frozen) ? 1 : 0;
    nact += act[d];
  }
  const int64_t npts = bst[0] * bx.m[0];
  const int64_t A = (int64_t)1 << a.L;
  // anchors
  for (int64_t i = threadIdx.x; i < npts; i += blockDim.x) {
    int64_t x[4];
    int64_t rr = i;
    bool anc = true;
    for (int d = 3; d >= 0; d--) {
      x[d] = rr % bx.m[d];
      rr /= bx.m[d];
      if (act[d] && x[d] % A != 0) anc = false;
    }
    if (anc) {
      const int64_t fidx = (bx.o[0] + x[0]) * a.fg.st[0] + (bx.o[1] + x[1]) * a.fg.st[1] +
                           (bx.o[2] + x[2]) * a.fg.st[2] + (bx.o[3] + x[3]);
      W[i] = X[fidx];
    }
  }
  __syncthreads();
  unsigned long long total_score = 0, sq = 0;
  for (int l = a.L; l >= 1; l--) {
    const int64_t s = (int64_t)1 << (l - 1);
    const hpez_interp ip = a.tuned ? a.level[l - 1] : a.cand[cand];
    unsigned long long sc = 0;
    int64_t r[4], m[4];
    if (ip.md) {
      for (int cnt = 1; cnt <= nact; cnt++) {
        for (unsigned odd = 1; odd < 16; odd++) {
          bool ok = __popc(odd) == cnt;
          for (int d = 0; d < 4; d++)
            if ((odd >> d & 1u) && !act[d]) ok = false;
          if (!ok) continue;
          for (int d = 0; d < 4; d++) {
            if (!act[d]) { r[d] = 0; m[d] = 1; }
            else if (odd >> d & 1u) { r[d] = s; m[d] = 2 * s; }
            else { r[d] = 0; m[d] = 2 * s; }
          }
          trial_step<T, P>(a, bx, bst, X, W, r, m, ip.kind, 1, 0, -1, odd, s, l, wq, sc, hist, lh, sq);
        }
        __syncthreads();
      }
    } else {
      // pass position of each dim, 4 bits per dim (15: not in the pass order)
      unsigned pos = 0xffffu;
      int np = 0;
      for (int i = 0; i < 4; i++) {
        const int d = ip.order[i];
        bool fresh = false;
        for (int e = 0; e < 4; e++)
          if (e == d && act[e] && (pos >> (4 * e) & 15u) == 15u) fresh = true;
        if (fresh) pos = (pos & ~(15u << (4 * d))) | ((unsigned)np++ << (4 * d));
      }
      for (int k = 0; k < np; k++) {
        int pd = 0;
        for (int d = 0; d < 4; d++)
          if ((pos >> (4 * d) & 15u) == (unsigned)k) pd = d;
        for (int d = 0; d < 4; d++) {
          const unsigned pdd = pos >> (4 * d) & 15u;
          if (!act[d]) { r[d] = 0; m[d] = 1; }
          else if (d == pd) { r[d] = s; m[d] = 2 * s; }
          else if (pdd == 15u || pdd < (unsigned)k) { r[d] = 0; m[d] = s; }
          else { r[d] = 0; m[d] = 2 * s; }
        }
        if (ip.kind != 0 && ip.same_level) {
          for (int d = 0; d < 4; d++)
            if (d == pd) {
              m[d] = 4 * s;
              r[d] = s;
            }
          trial_step<T, P>(a, bx, bst, X, W, r, m, ip.kind, 0, 0, pd, 0, s, l, wq, sc, hist, lh, sq);
          __syncthreads();
          for (int d = 0; d < 4; d++)
            if (d == pd) r[d] = 3 * s;
          trial_step<T, P>(a, bx, bst, X, W, r, m, ip.kind, 0, 1, pd, 0, s, l, wq, sc, hist, lh, sq);
        } else {
          trial_step<T, P>(a, bx, bst, X, W, r, m, ip.kind, 0, 0, pd, 0, s, l, wq, sc, hist, lh, sq);
        }
        __syncthreads();
      }
    }
    const unsigned long long v = block_sum_u64(sc, red);
    if (a.score_mode == 0) {
      if (threadIdx.x == 0 && v) atomicAdd(&score[cand * 16 + (l - 1)], v);
    } else {
      total_score += v;
    }
  }
  if (a.score_mode == 1 && threadIdx.x == 0) score[(uint64_t)blockIdx.x * gridDim.y + cand] = total_score;
  if (a.score_mode == 2) {
    const unsigned long long v = block_sum_u64(sq, red);
    if (threadIdx.x == 0 && v) atomicAdd(&score[0], v);
  }
  if (hist) {
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < kTrialHistWin; i += blockDim.x)
      if (lh[i]) atomicAdd(&hist[a.hist_lo + i], lh[i]);
  }
}

// regions too large for LDS: the region's working copy in global scratch,
// 1024 lanes per (region, candidate) (few work-groups, each a long serial
// walk through the levels)
constexpr int kTrialGlobalThreads = 1024;

template <typename T>
__global__ void __launch_bounds__(kTrialGlobalThreads) trial_kernel_global(TrialArgs a,
                                                           const TrialBox* __restrict__ boxes,
                                                           const T* __restrict__ X,
                                                           T* __restrict__ scratch,
                                                           const double* __restrict__ wq,
                                                           unsigned long long* __restrict__ score,
                                                           uint32_t* __restrict__ hist)
{
  extern __shared__ unsigned char lds_raw[];
  const TrialBox bx = boxes[blockIdx.x];
  T* W = scratch + ((uint64_t)blockIdx.x * gridDim.y + blockIdx.y) * a.box_cap;
  trial_body<T, T>(a, bx, X, W, (int)blockIdx.y, wq, score, hist,
                   reinterpret_cast<uint32_t*>(lds_raw));
}

template <typename T>
__global__ void __launch_bounds__(256) trial_kernel_lds(TrialArgs a,
                                                        const TrialBox* __restrict__ boxes,
                                                        const T* __restrict__ X,
                                                        const double* __restrict__ wq,
                                                        unsigned long long* __restrict__ score,
                                                        uint32_t* __restrict__ hist)
{
  extern __shared__ unsigned char lds_raw[];
  T* W = reinterpret_cast<T*>(lds_raw);
  const TrialBox bx = boxes[blockIdx.x];
  trial_body<T, T>(a, bx, X, W, (int)blockIdx.y, wq, score, hist,
                   reinterpret_cast<uint32_t*>(lds_raw + ((a.box_cap * sizeof(T) + 15) & ~15ull)));
}

// per-point work of a trial: score the prediction error, quantize, write the
// reconstruction back (and count the code)
template <typename T, bool HIST>
struct TrialOp {
  using Fetched = int;
  T* L;
  uint32_t* lh;
  HPEZ_GLOBAL uint32_t* hist;
  uint32_t R, lo;
  double el, inv2e, twoe, mul;
  unsigned long long sc;
  uint32_t nR;
  double inv_e;  // > 0: accumulate the distortion of Sec. 6.4 into sq
  unsigned long long sq;
  __device__ __forceinline__ int fetch(int32_t, int32_t, int32_t, bool) const { return 0; }
  __device__ __forceinline__ void apply(int32_t li, int32_t, int32_t, int32_t, T p, int)
  {
    const T xv = L[li];
    const double t = fabs((double)xv - (double)p) * mul;
    // below 2^32 the floor converts exactly through 32 bits
    sc += (t < 4294967296.0) ? (unsigned long long)(uint32_t)floor(t) : 4294967296ull;
    T xr = xv;
    const uint32_t q = quantize<T>(xv, p, inv2e, twoe, el, R, xr);
    L[li] = xr;
    if (inv_e > 0.0) {
      const double u = ((double)xv - (double)xr) * inv_e;
      sq += (unsigned long long)floor(u * u * 4294967296.0);
    }
    if (HIST) {
      nR += q == R;
      if (q != R) {
        const uint32_t w = q - lo;
        if (w < kTrialHistWin)
          __hip_atomic_fetch_add(&lh[w], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else
          __hip_atomic_fetch_add(&hist[q], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
};

// Trial of a region of at most three dims held entirely in LDS (original
// values, then reconstructions in place), on the shared box schedule.  The
// region is tb (index ib of n_cand-wide score rows), the candidate cand.
template <typename T, bool HIST, int NT>
__device__ __forceinline__ void trial_box_run(const TrialArgs& a, const TrialBox& tb, uint32_t ib,
                                              int cand, uint32_t n_cand,
                                              const HPEZ_GLOBAL T* __restrict__ X,
                                              HPEZ_GLOBAL unsigned long long* __restrict__ score,
                                              HPEZ_GLOBAL uint32_t* __restrict__ hist,
                                              unsigned char* lds_raw, unsigned long long* red)
{
  T* L = reinterpret_cast<T*>(lds_raw);
  uint32_t* lh = reinterpret_cast<uint32_t*>(lds_raw + ((a.box_cap * sizeof(T) + 15) & ~15ull));
  const int32_t frozen = a.frozen;
  Box bx;
  bx.E0 = (int32_t)tb.m[0];
  bx.E1 = (int32_t)tb.m[1];
  bx.E2 = (int32_t)tb.m[2];
  bx.b1 = bx.E2;
  bx.b0 = bx.E1 * bx.E2;
  bx.a0 = bx.E0 > 1 && frozen != 0;
  bx.a1 = bx.E1 > 1 && frozen != 1;
  bx.a2 = bx.E2 > 1 && frozen != 2;
  bx.lo0 = bx.lo1 = bx.lo2 = 0;
  bx.hi0 = bx.E0 - 1;
  bx.hi1 = bx.E1 - 1;
  bx.hi2 = bx.E2 - 1;
  // the region, row-major
  const uint32_t npts = (uint32_t)bx.E0 * bx.b0;
  const Divisor mgb0 = fmagic((uint32_t)bx.b0);
  const Divisor mgE2 = fmagic((uint32_t)bx.E2);
  const int64_t st0 = a.fg.st[0], st1 = a.fg.st[1];
  const HPEZ_GLOBAL T* __restrict__ Xo = X + tb.o[0] * st0 + tb.o[1] * st1 + tb.o[2];
  for (uint32_t i = threadIdx.x; i < npts; i += NT) {
    const uint32_t c0 = fdiv(i, mgb0);
    const uint32_t rem = i - c0 * (uint32_t)bx.b0;
    const uint32_t c1 = fdiv(rem, mgE2);
    const uint32_t c2 = rem - c1 * (uint32_t)bx.E2;
    L[i] = Xo[c0 * st0 + c1 * st1 + c2];
  }
  const uint32_t R = a.R, hist_lo = a.hist_lo;
  if (HIST)
    for (uint32_t i = threadIdx.x; i < kTrialHistWin; i += NT) lh[i] = 0;
  __syncthreads();
  unsigned long long total_score = 0, total_sq = 0;
  uint32_t nR = 0;
  const int score_mode = a.score_mode;
  for (int l = a.L; l >= 1; l--) {
    const int32_t s = 1 << (l - 1);
    const hpez_interp ip = a.tuned ? a.level[l - 1] : a.cand[cand];
    TrialOp<T, HIST> op{L,           lh,        hist,        R,    hist_lo, a.el[l],
                        a.inv2e[l],  a.twoe[l], a.score_mul, 0ull, 0u,
                        score_mode == 2 ? a.inv_e : 0.0, 0ull};
    box_level<T, NT>(ip, bx, L, 0, 0, 0, s, a.wmd, op);
    nR += op.nR;
    total_sq += op.sq;
    const unsigned long long v = block_sum_u64(op.sc, red);
    if (score_mode == 0) {
      if (threadIdx.x == 0 && v)
        __hip_atomic_fetch_add(&score[cand * 16 + (l - 1)], v, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    } else {
      total_score += v;
    }
  }
  if (score_mode == 1 && threadIdx.x == 0) score[(uint64_t)ib * n_cand + cand] = total_score;
  if (score_mode == 2) {
    const unsigned long long v = block_sum_u64(total_sq, red);
    if (threadIdx.x == 0 && v)
      __hip_atomic_fetch_add(&score[0], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (HIST) {
    for (int o = 32; o > 0; o >>= 1) nR += __shfl_xor(nR, o, 64);
    if ((threadIdx.x & 63) == 0 && nR) {
      const uint32_t w = R - hist_lo;
      if (w < kTrialHistWin) atomicAdd(&lh[w], nR);
      else __hip_atomic_fetch_add(&hist[R], nR, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < kTrialHistWin; i += NT)
      if (lh[i])
        __hip_atomic_fetch_add(&hist[hist_lo + i], lh[i], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename T, bool HIST, int NT>
__global__ void __launch_bounds__(NT) trial_box_kernel(TrialArgs a, const TrialBox* __restrict__ boxes,
                                                       const T* __restrict__ X,
                                                       unsigned long long* __restrict__ score,
                                                       uint32_t* __restrict__ hist)
{
  extern __shared__ unsigned char lds_raw[];
  __shared__ unsigned long long red[16];
  trial_box_run<T, HIST, NT>(a, boxes[blockIdx.x], blockIdx.x, (int)blockIdx.y, gridDim.y, gmem(X),
                             gmem(score), gmem(hist), lds_raw, red);
}

// index of the last entry whose begin is <= x (begin ascending, begin[0] = 0)
__device__ __forceinline__ int trial_entry(const uint64_t* __restrict__ begin, int n, uint64_t x)
{
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Every (region, candidate) trial of several tuning runs (fields, freeze
// variants) in one launch: work-group w belongs to the entry whose range of
// n_boxes * n_cand work-groups holds it.
template <typename T, bool HIST, int NT>
__global__ void __launch_bounds__(NT) trial_jobs_kernel(const TrialJob<T>* __restrict__ jobs,
                                                        const uint64_t* __restrict__ wg_begin, int n)
{
  extern __shared__ unsigned char lds_raw[];
  __shared__ unsigned long long red[16];
  const int j = trial_entry(wg_begin, n, blockIdx.x);
  const TrialJob<T>& J = jobs[j];
  const uint32_t nc = J.n_cand;
  const uint32_t local = (uint32_t)(blockIdx.x - J.wg_begin);
  const uint32_t ib = local / nc;
  const int cand = (int)(local - ib * nc);
  trial_box_run<T, HIST, NT>(J.a, J.boxes[ib], ib, cand, nc, gmem(J.X), gmem(J.score),
                             gmem(J.hist), lds_raw, red);
}

template <typename T>
bool trial_box_ok(const TrialArgs& a, bool hist)
{
  const size_t box = (size_t)a.box_cap * sizeof(T);
  const size_t lds_all = ((box + 15) & ~(size_t)15) + (hist ? (size_t)kTrialHistWin * 4 : 0);
  return a.fg.n[3] == 1 && lds_all <= kTrialBoxLdsBytes && a.box_cap < 65536 &&
         (uint64_t)a.max_ext * (uint64_t)a.max_ext <= kMagicMax;
}

template <typename T>
size_t trial_box_lds(const TrialArgs& a, bool hist)
{
  const size_t box = (size_t)a.box_cap * sizeof(T);
  return ((box + 15) & ~(size_t)15) + (hist ? (size_t)kTrialHistWin * 4 : 0);
}

template <typename T, bool HIST, int NT>
static void launch_jobs_t(const TrialJob<T>* d_jobs, const uint64_t* d_wg_begin, int n,
                          uint64_t total_wg, size_t lds, hipStream_t st)
{
  (void)hipFuncSetAttribute((const void*)trial_jobs_kernel<T, HIST, NT>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((trial_jobs_kernel<T, HIST, NT>), dim3((unsigned)total_wg), dim3(NT), lds, st,
                     d_jobs, d_wg_begin, n);
}

template <typename T>
hipError_t launch_trial_jobs(const TrialJob<T>* d_jobs, const uint64_t* d_wg_begin, int n,
                             uint64_t total_wg, size_t lds, bool hist, int lanes, hipStream_t st)
{
  if (!total_wg || n <= 0) return hipSuccess;
  if (hist && lanes == 1024) launch_jobs_t<T, true, 1024>(d_jobs, d_wg_begin, n, total_wg, lds, st);
  else if (hist && lanes == 256) launch_jobs_t<T, true, 256>(d_jobs, d_wg_begin, n, total_wg, lds, st);
  else if (hist) launch_jobs_t<T, true, 64>(d_jobs, d_wg_begin, n, total_wg, lds, st);
  else if (lanes == 1024) launch_jobs_t<T, false, 1024>(d_jobs, d_wg_begin, n, total_wg, lds, st);
  else if (lanes == 256) launch_jobs_t<T, false, 256>(d_jobs, d_wg_begin, n, total_wg, lds, st);
  else launch_jobs_t<T, false, 64>(d_jobs, d_wg_begin, n, total_wg, lds, st);
  return hipGetLastError();
}

template <typename T, bool HIST, int NT>
static void launch_box_trials(const TrialArgs& a, const TrialBox* d_boxes, uint32_t n_boxes,
                              uint32_t n_cand, const T* X, unsigned long long* d_score,
                              uint32_t* d_hist, size_t lds, hipStream_t st)
{
  (void)hipFuncSetAttribute((const void*)trial_box_kernel<T, HIST, NT>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((trial_box_kernel<T, HIST, NT>), dim3(n_boxes, n_cand), dim3(NT), lds, st, a,
                     d_boxes, X, d_score, d_hist);
}

template <typename T>
hipError_t launch_trials(const TrialArgs& a, const TrialBox* d_boxes, uint32_t n_boxes,
                         uint32_t n_cand, const T* X, T* scratch, const double* d_wq,
                         unsigned long long* d_score, uint32_t* d_hist, hipStream_t st)
{
  if (!n_boxes || !n_cand) return hipSuccess;
  const size_t box = (size_t)a.box_cap * sizeof(T);
  const size_t hb = d_hist ? (size_t)kTrialHistWin * 4 : 0;
  const size_t lds_all = ((box + 15) & ~(size_t)15) + hb;
  // in-LDS regions: at most three dims, index arithmetic within the constant
  // divisor table (every product of two extents <= kMagicMax) and 16 bits
  if (a.fg.n[3] == 1 && lds_all <= kTrialBoxLdsBytes && a.box_cap < 65536 &&
      (uint64_t)a.max_ext * (uint64_t)a.max_ext <= kMagicMax) {
    // regions of at most three dims in LDS: 1024 lanes for large regions
    const bool big = a.box_cap > 4096;
    if (d_hist && big)
      launch_box_trials<T, true, 1024>(a, d_boxes, n_boxes, n_cand, X, d_score, d_hist, lds_all, st);
    else if (d_hist)
      launch_box_trials<T, true, 256>(a, d_boxes, n_boxes, n_cand, X, d_score, d_hist, lds_all, st);
    else if (big)
      launch_box_trials<T, false, 1024>(a, d_boxes, n_boxes, n_cand, X, d_score, d_hist, lds_all, st);
    else
      launch_box_trials<T, false, 256>(a, d_boxes, n_boxes, n_cand, X, d_score, d_hist, lds_all, st);
    return hipGetLastError();
  }
  if (box <= kTrialLdsBytes) {
    const size_t lds = ((box + 15) & ~(size_t)15) + hb;
    (void)hipFuncSetAttribute((const void*)trial_kernel_lds<T>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((trial_kernel_lds<T>), dim3(n_boxes, n_cand), dim3(256), lds, st, a,
                       d_boxes, X, d_wq, d_score, d_hist);
  } else
    hipLaunchKernelGGL((trial_kernel_global<T>), dim3(n_boxes, n_cand), dim3(kTrialGlobalThreads),
                       hb, st, a, d_boxes, X, scratch, d_wq, d_score, d_hist);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Lorenzo trial: dual-quantized first-order residuals of every region point
template <typename T>
__global__ void __launch_bounds__(256) lorenzo_trial_kernel(Geom fg, const TrialBox* __restrict__ boxes,
                                                            const T* __restrict__ X, double inv2e,
                                                            uint32_t R, uint32_t hist_lo,
                                                            uint32_t* __restrict__ hist,
                                                            int* __restrict__ unsupported)
{
  __shared__ uint32_t lh[kTrialHistWin];
  for (uint32_t i = threadIdx.x; i < kTrialHistWin; i += blockDim.x) lh[i] = 0;
  __syncthreads();
  const TrialBox bx = boxes[blockIdx.y];
  const int64_t st0 = fg.st[0], st1 = fg.st[1], st2 = fg.st[2];
  const int64_t sd[4] = {st0, st1, st2, 1};
  // one point: its Lorenzo residual (sum over the corners of the unit cell
  // behind it, each stepping back one along the dims of S) into the histogram
  auto point = [&](const int64_t* x) {
    const int64_t base = (bx.o[0] + x[0]) * st0 + (bx.o[1] + x[1]) * st1 +
                         (bx.o[2] + x[2]) * st2 + (bx.o[3] + x[3]);
    long long delta = 0;
    bool bad = false;
    for (unsigned S = 0; S < 16; S++) {
      bool in = true;
      int64_t fidx = base;
      for (int d = 0; d < 4; d++)
        if ((S >> d) & 1u) {
          if (x[d] == 0) in = false;
          fidx -= sd[d];
        }
      if (!in) continue;
      const double t = (double)X[fidx] * inv2e;
      const double qf = floor(fabs(t) + 0.5);
      if (!(qf < 4503599627370496.0)) {
        bad = true;
        continue;
      }
      const long long v = (long long)(t < 0 ? -qf : qf);
      delta += (__popc(S) & 1) ? -v : v;
    }
    if (bad) {
      atomicOr(unsupported, 1);
      return;
    }
    const uint32_t code = (delta > -(long long)R && delta < (long long)R) ? (uint32_t)(delta + R) : 0u;
    hist_add_wave(lh, hist, hist_lo, kTrialHistWin, code, true);
  };
  const uint64_t np = (uint64_t)bx.m[0] * bx.m[1] * bx.m[2] * bx.m[3];
  if (np <= (1ull << 31)) {
    // 32-bit coordinates by exact multiply-high division (index + grid stride
    // stays below 2^32)
    const uint32_t npts = (uint32_t)np;
    const uint32_t m1 = (uint32_t)bx.m[1], m2 = (uint32_t)bx.m[2], m3 = (uint32_t)bx.m[3];
    const XDivisor d1 = xmagic(m1), d2 = xmagic(m2), d3 = xmagic(m3);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += gridDim.x * blockDim.x) {
      const uint32_t q3 = xdiv(i, d3), x3 = i - q3 * m3;
      const uint32_t q2 = xdiv(q3, d2), x2 = q3 - q2 * m2;
      const uint32_t x0 = xdiv(q2, d1), x1 = q2 - x0 * m1;
      const int64_t x[4] = {x0, x1, x2, x3};
      point(x);
    }
  } else {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np;
         i += (uint64_t)gridDim.x * blockDim.x) {
      int64_t x[4];
      uint64_t rr = i;
      for (int d = 3; d >= 0; d--) {
        x[d] = (int64_t)(rr % (uint64_t)bx.m[d]);
        rr /= (uint64_t)bx.m[d];
      }
      point(x);
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < kTrialHistWin; i += blockDim.x)
    if (lh[i]) atomicAdd(&hist[hist_lo + i], lh[i]);
}

template <typename T>
hipError_t launch_lorenzo_trial(const Geom& fg, const TrialBox* d_boxes, uint32_t n_boxes,
                                uint32_t max_pts, const T* X, double inv2e, uint32_t R,
                                uint32_t hist_lo, uint32_t* d_hist, int* d_unsupported,
                                hipStream_t st)
{
  if (!n_boxes) return hipSuccess;
  // a few work-groups per region, each walking many points, so the LDS
  // histogram is flushed rarely
  unsigned gx = (max_pts + 255) / 256;
  if (gx > 8) gx = 8;
  hipLaunchKernelGGL((lorenzo_trial_kernel<T>), dim3(gx ? gx : 1, n_boxes), dim3(256), 0, st, fg,
                     d_boxes, X, inv2e, R, hist_lo, d_hist, d_unsupported);
  return hipGetLastError();
}

// histogram blockIdx.y of a set: its bins at hist + y nsym, its count at
// count[y], its pairs at pairs + y 2 cap
__global__ void __launch_bounds__(256) hist_nonzero_kernel(const uint32_t* __restrict__ hist,
                                                           uint32_t nsym, uint32_t* __restrict__ count,
                                                           uint32_t* __restrict__ pairs, uint32_t cap)
{
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nsym) return;
  hist += (size_t)blockIdx.y * nsym;
  count += blockIdx.y;
  pairs += (size_t)blockIdx.y * 2 * cap;
  const uint32_t c = hist[k];
  if (!c) return;
  const uint32_t i = atomicAdd(count, 1u);
  if (i < cap) {
    pairs[2 * i] = k;
    pairs[2 * i + 1] = c;
  }
}

hipError_t launch_hist_nonzero(const uint32_t* d_hist, uint32_t nsym, uint32_t* d_count,
                               uint32_t* d_pairs, uint32_t cap, hipStream_t st)
{
  if (!nsym) return hipSuccess;
  hipLaunchKernelGGL(hist_nonzero_kernel, dim3((nsym + 255) / 256), dim3(256), 0, st, d_hist, nsym,
                     d_count, d_pairs, cap);
  return hipGetLastError();
}

hipError_t launch_hist_nonzero_set(const uint32_t* d_hist, uint32_t nsym, uint32_t n,
                                   uint32_t* d_count, uint32_t* d_pairs, uint32_t cap,
                                   hipStream_t st)
{
  if (!nsym || !n) return hipSuccess;
  hipLaunchKernelGGL(hist_nonzero_kernel, dim3((nsym + 255) / 256, n), dim3(256), 0, st, d_hist,
                     nsym, d_count, d_pairs, cap);
  return hipGetLastError();
}

#define INST(T)                                                                                 \
  template hipError_t launch_stats<T>(const T*, const Geom&, const Lattice&, double,            \
                                      unsigned long long*, hipStream_t);                        \
  template hipError_t launch_trial_jobs<T>(const TrialJob<T>*, const uint64_t*, int, uint64_t,     \
                                           size_t, bool, int, hipStream_t);                      \
  template bool trial_box_ok<T>(const TrialArgs&, bool);                                         \
  template size_t trial_box_lds<T>(const TrialArgs&, bool);                                      \
  template hipError_t launch_trials<T>(const TrialArgs&, const TrialBox*, uint32_t, uint32_t,   \
                                       const T*, T*, const double*, unsigned long long*,        \
                                       uint32_t*, hipStream_t);                                 \
  template hipError_t launch_lorenzo_trial<T>(const Geom&, const TrialBox*, uint32_t, uint32_t, \
                                              const T*, double, uint32_t, uint32_t, uint32_t*,  \
                                              int*, hipStream_t);
INST(float)
INST(double)

}  // namespace hpez
