// k_interp.hip -- interpolation predictor kernels (gfx950).
//
// Level-wise anchor-based interpolation (Sec. 5.1) with linear-scale
// quantization (Sec. 4, step 3): for each level, each step (one 1D pass, one
// half of a same-level split pass, or one multi-dimensional sub-step) is one
// launch over exactly the points that step predicts.  Each thread predicts one
// point from already reconstructed neighbours in W, quantizes the error
// (compress) or applies the decoded code (decompress), and writes the
// reconstruction back to W.  Points of one step never read each other, so the
// traversal order inside a launch does not matter (Sec. 5.4.1); lanes map to
// the fastest-varying dimension so that reads and writes coalesce.
//
// Floating point: the stencils are evaluated in T in the order written, the
// quantizer in double; the library is built with -ffp-contract=off so no
// operation is fused.

#include "interp_dev.h"

namespace hpez {

template <typename T, int MODE>
__device__ __forceinline__ void finish(T p, int64_t idx, int64_t cpos, const T* __restrict__ X,
                                       T* __restrict__ W, uint16_t* __restrict__ code, double el,
                                       double inv2e, double twoe, uint32_t R)
{
  if (MODE == 0) {
    const T x = X[idx];
    T xr = x;
    const uint32_t q = quantize<T>(x, p, inv2e, twoe, el, R, xr);
    code[cpos] = (uint16_t)q;
    W[idx] = q ? xr : x;
  } else {
    const uint32_t q = code[cpos];
    if (q != 0) W[idx] = recon<T>(p, (double)((int32_t)q - (int32_t)R), twoe);
  }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(256) step_kernel(StepArgs a, const T* __restrict__ X,
                                                   T* __restrict__ W, uint16_t* __restrict__ code)
{
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t total = a.filter ? a.fstart[a.nface] : a.lat.total;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += stride) {
    int64_t x[4];
    if (a.filter) {
      // a point on several faces is taken by its first face dim only
      int f = 0;
      while (f + 1 < a.nface && k >= a.fstart[f + 1]) f++;
      lattice_point(a.flat[f], k - a.fstart[f], x);
      bool earlier = false;
      for (int d = 0; d < 4; d++)
        if (d < a.fdim[f] && a.g.act[d] && (x[d] & (a.B - 1)) == 0) earlier = true;
      if (earlier) continue;
    } else {
      lattice_point(a.lat, k, x);
    }
    if (a.md && a.mdhalf && md_colour(x, a.odd, a.s) != a.mdhalf - 1) continue;
    const int64_t idx = x[0] * a.g.st[0] + x[1] * a.g.st[1] + x[2] * a.g.st[2] + x[3];
    T p;
    if (!a.md) {
      const int d = a.pdim;
      p = spline<T, T>(W, idx, a.s * a.g.st[d], x[d], a.s, 0, a.g.n[d] - 1, a.kind, a.sl);
    } else {
      bool first = true;
      T acc = (T)0;
      for (int d = 0; d < 4; d++) {
        if (!(a.odd >> d & 1u)) continue;
        const T pd = spline<T, T>(W, idx, a.s * a.g.st[d], x[d], a.s, 0, a.g.n[d] - 1, a.kind, a.sl);
        const T term = (T)a.wq[d] * pd;
        acc = first ? term : acc + term;
        first = false;
      }
      p = acc;
    }
    finish<T, MODE>(p, idx, brick_pos(a.g.n, x), X, W, code, a.el, a.inv2e, a.twoe, a.R);
  }
}

// Step index of a level point under a configuration: 1D style, 2 * pass + half
// (the pass is the last dimension in pass order whose coordinate is an odd
// multiple of s; the half is 1 for coordinates at 3s mod 4s with same-level
// cubic); multi-dimensional, 2 * (number of odd coordinates - 1) + half (the
// half is the checkerboard colour with same-level cubic).  The stride s = 2^ls
// is a power of two and coordinates are nonnegative, so x / s is x >> ls.
__device__ __forceinline__ int step_of(const hpez_interp& c, const int32_t* act, const int64_t* x,
                                       int ls, unsigned* odd_out, int* pdim_out, int* half_out)
{
  unsigned odd = 0;
  for (int d = 0; d < 4; d++)
    if (act[d] && (x[d] >> ls) & 1) odd |= 1u << d;
  *odd_out = odd;
  if (c.md) {
    *pdim_out = -1;
    int half = 0;
    if (c.kind != 0 && c.same_level) {
      int64_t t = 0;
      for (int d = 0; d < 4; d++)
        if (odd >> d & 1u) t += x[d] >> (ls + 1);
      half = (int)(t & 1);
    }
    *half_out = half;
    return 2 * (__popc(odd) - 1) + half;
  }
  int pass = -1, pd = -1, k = 0;
  unsigned seen = 0, actm = 0;
  for (int d = 0; d < 4; d++)
    if (act[d]) actm |= 1u << d;
  for (int i = 0; i < 4; i++) {
    const int d = c.order[i];
    if (d < 4 && (actm >> d & 1u) && !(seen >> d & 1u)) {
      seen |= 1u << d;
      if (odd >> d & 1u) {
        pass = k;
        pd = d;
      }
      k++;
    }
  }
  *pdim_out = pd;
  const int half = (c.kind != 0 && c.same_level && ((pick4(x, pd) >> ls) & 3) == 3) ? 1 : 0;
  *half_out = half;
  return 2 * pass + half;
}

// Per-dim coordinate classes of a block's points at one level: every j in
// [1, J] (any), odd j, even j; x = lo + j s.  Frozen and size-1 dims take
// every coordinate lo + j, j in [0, J).
enum : int { kJAny = 0, kJOdd = 1, kJEven = 2 };

// Interior points of every block at one level, one step index of each block's
// own configuration.  A step's points inside one block form at most six
// product sets of per-dim progressions: a 1D pass has its pass dim odd, the
// dims before it in pass order anything and the dims after it even; a
// multi-dimensional sub-step with c odd dims has one set per choice of c odd
// active dims.  One work-group takes one of `pieces` parts of one block: its
// first lane lays the block's sets out in LDS, the lanes walk their points,
// and the step test (which also splits same-level halves and checkerboard
// colours) keeps exactly the step's points.  A block's extent along an
// active dim is below B, so its lower corner is an even multiple of s and the
// parity of x / s is the parity of j.
template <typename T, int MODE>
__global__ void __launch_bounds__(256) block_step_kernel(BlockStepArgs a, const T* __restrict__ X,
                                                         T* __restrict__ W,
                                                         uint16_t* __restrict__ code,
                                                         const uint8_t* __restrict__ bcfg,
                                                         const double* __restrict__ wq)
{
  __shared__ uint32_t s_first[6][4], s_step[6][4], s_cnt[6][4];
  __shared__ uint64_t s_start[7];
  __shared__ int s_nbox;
  const int ls = __builtin_ctzll((unsigned long long)a.s);
  const uint64_t nbt = (uint64_t)a.nb[0] * a.nb[1] * a.nb[2] * a.nb[3];
  const uint32_t P = a.pieces;
  for (uint64_t u = blockIdx.x; u < nbt * P; u += gridDim.x) {
    const uint64_t bi = u / P;
    const uint32_t piece = (uint32_t)(u - bi * P);
    const hpez_interp c = a.cand[bcfg[bi]];
    // second halves exist only with same-level cubic (uniform: no barrier)
    if ((a.t & 1) && !(c.kind != 0 && c.same_level)) continue;
    int64_t lo[4], hi[4], J[4];
    {
      uint64_t r = bi;
      for (int d = 3; d >= 0; d--) {
        const uint64_t q = r / (uint64_t)a.nb[d];
        lo[d] = (int64_t)(r - q * (uint64_t)a.nb[d]) * a.B;
        r = q;
      }
    }
    for (int d = 0; d < 4; d++) {
      hi[d] = lo[d] + a.B < a.g.n[d] - 1 ? lo[d] + a.B : a.g.n[d] - 1;
      const int64_t top = lo[d] + a.B - 1 < a.g.n[d] - 1 ? lo[d] + a.B - 1 : a.g.n[d] - 1;
      J[d] = a.g.act[d] ? (top - lo[d]) >> ls : top - lo[d] + 1;
    }
    if (threadIdx.x == 0) {
      // progression of dim d in set bx for class cl; returns its length
      auto put = [&](int bx, int d, int cl) -> uint64_t {
        uint32_t f = 1, st = 1, n = (uint32_t)J[d];
        if (!a.g.act[d]) {
          f = 0;
        } else if (cl == kJOdd) {
          st = 2;
          n = (uint32_t)((J[d] + 1) >> 1);
        } else if (cl == kJEven) {
          f = 2;
          st = 2;
          n = (uint32_t)(J[d] >> 1);
        }
        s_first[bx][d] = f;
        s_step[bx][d] = st;
        s_cnt[bx][d] = n;
        return n;
      };
      int nbox = 0;
      uint64_t run = 0;
      const bool halves = c.kind != 0 && c.same_level;
      if (!(a.t & 1) || halves) {
        if (c.md) {
          const int want = (a.t >> 1) + 1;
          for (unsigned odd = 1; odd < 16 && nbox < 6; odd++) {
            bool ok = (int)__popc(odd) == want;
            for (int d = 0; d < 4; d++)
              if ((odd >> d & 1u) && !a.g.act[d]) ok = false;
            if (!ok) continue;
            s_start[nbox] = run;
            uint64_t prod = 1;
            for (int d = 0; d < 4; d++) prod *= put(nbox, d, (odd >> d & 1u) ? kJOdd : kJEven);
            run += prod;
            nbox++;
          }
        } else {
          // pass position of each dim, 4 bits per dim (15: not in the pass order)
          unsigned pos = 0xffffu, actm = 0;
          int np = 0;
          for (int d = 0; d < 4; d++)
            if (a.g.act[d]) actm |= 1u << d;
          for (int i = 0; i < 4; i++) {
            const int d = c.order[i];
            if (d < 4 && (actm >> d & 1u) && (pos >> (4 * d) & 15u) == 15u)
              pos = (pos & ~(15u << (4 * d))) | ((unsigned)np++ << (4 * d));
          }
          const int k = a.t >> 1;
          if (k < np) {
            s_start[0] = 0;
            uint64_t prod = 1;
            for (int d = 0; d < 4; d++) {
              const unsigned pd = pos >> (4 * d) & 15u;
              prod *= put(0, d, pd == (unsigned)k ? kJOdd
                                : pd != 15u && pd > (unsigned)k ? kJEven
                                                                : kJAny);
            }
            run = prod;
            nbox = 1;
          }
        }
      }
      s_start[nbox] = run;
      s_nbox = nbox;
    }
    __syncthreads();
    const int nbox = s_nbox;
    const uint64_t total = s_start[nbox];
    const bool narrow = total <= 0xffffffffull;
    for (uint64_t k = (uint64_t)piece * blockDim.x + threadIdx.x; k < total;
         k += (uint64_t)P * blockDim.x) {
      int bx = 0;
      while (bx + 1 < nbox && k >= s_start[bx + 1]) bx++;
      int64_t x[4];
      if (narrow) {
        uint32_t r = (uint32_t)(k - s_start[bx]);
        for (int d = 3; d >= 0; d--) {
          const uint32_t n = s_cnt[bx][d];
          const uint32_t q = r / n;
          const int64_t j = (int64_t)s_first[bx][d] + (int64_t)s_step[bx][d] * (r - q * n);
          x[d] = lo[d] + (a.g.act[d] ? j << ls : j);
          r = q;
        }
      } else {
        uint64_t r = k - s_start[bx];
        for (int d = 3; d >= 0; d--) {
          const uint64_t n = s_cnt[bx][d];
          const uint64_t q = r / n;
          const int64_t j = (int64_t)s_first[bx][d] + (int64_t)s_step[bx][d] * (int64_t)(r - q * n);
          x[d] = lo[d] + (a.g.act[d] ? j << ls : j);
          r = q;
        }
      }
      unsigned odd;
      int pd, half;
      if (step_of(c, a.g.act, x, ls, &odd, &pd, &half) != a.t) continue;
      const int64_t idx = x[0] * a.g.st[0] + x[1] * a.g.st[1] + x[2] * a.g.st[2] + x[3];
      T p;
      if (!c.md) {
        p = spline<T, T>(W, idx, a.s * pick4(a.g.st, pd), pick4(x, pd), a.s, pick4(lo, pd),
                         pick4(hi, pd), c.kind, half);
      } else {
        bool first = true;
        T acc = (T)0;
        for (int d = 0; d < 4; d++) {
          if (!(odd >> d & 1u)) continue;
          const T pdv = spline<T, T>(W, idx, a.s * a.g.st[d], x[d], a.s, lo[d], hi[d], c.kind, half);
          const T term = (T)wq[(c.kind * 16 + odd) * 4 + d] * pdv;
          acc = first ? term : acc + term;
          first = false;
        }
        p = acc;
      }
      finish<T, MODE>(p, idx, brick_pos(a.g.n, x), X, W, code, a.el, a.inv2e, a.twoe, a.R);
    }
    __syncthreads();
  }
}

// Anchors (Sec. 5.1): kept verbatim, in row-major order.
template <typename T, int MODE>
__global__ void __launch_bounds__(256) anchor_kernel(Geom g, Lattice lat, const T* __restrict__ X,
                                                     T* __restrict__ W, uint16_t* __restrict__ code,
                                                     T* __restrict__ out_anchor, uint32_t R)
{
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < lat.total; k += stride) {
    int64_t x[4];
    lattice_point(lat, k, x);
    const int64_t idx = x[0] * g.st[0] + x[1] * g.st[1] + x[2] * g.st[2] + x[3];
    if (MODE == 0) {
      const T v = X[idx];
      W[idx] = v;
      code[brick_pos(g.n, x)] = (uint16_t)R;
      out_anchor[k] = v;
    } else {
      W[idx] = out_anchor[k];
    }
  }
}

static unsigned grid_for(uint64_t total)
{
  uint64_t b = (total + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// The points of lattice L whose coordinate along d is a multiple of B (a
// power of two): a sub-lattice along d, or none.
static bool face_lattice(const Lattice& L, int d, int64_t B, Lattice* out)
{
  const uint64_t cnt = L.cnt[d];
  uint64_t k0 = 0;
  while (k0 < cnt && k0 < (uint64_t)B && (L.first[d] + L.step[d] * (int64_t)k0) % B != 0) k0++;
  if (k0 >= cnt || k0 >= (uint64_t)B) return false;
  uint64_t dk = 1;
  while ((L.step[d] * (int64_t)dk) % B != 0) dk <<= 1;
  *out = L;
  out->first[d] = L.first[d] + L.step[d] * (int64_t)k0;
  out->step[d] = L.step[d] * (int64_t)dk;
  out->cnt[d] = (uint32_t)((cnt - 1 - k0) / dk + 1);
  out->total = 1;
  for (int e = 0; e < 4; e++) out->total *= out->cnt[e];
  return true;
}

template <typename T>
hipError_t launch_step(const StepArgs& a0, const T* X, T* W, uint16_t* code, int mode,
                       hipStream_t st)
{
  if (a0.lat.total == 0) return hipSuccess;
  StepArgs a = a0;
  uint64_t total = a.lat.total;
  if (a.filter) {
    a.nface = 0;
    a.fstart[0] = 0;
    for (int d = 0; d < 4; d++) {
      if (!a.g.act[d] || !face_lattice(a.lat, d, a.B, &a.flat[a.nface])) continue;
      a.fdim[a.nface] = d;
      a.fstart[a.nface + 1] = a.fstart[a.nface] + a.flat[a.nface].total;
      a.nface++;
    }
    total = a.fstart[a.nface];
    if (total == 0) return hipSuccess;
  }
  if (mode == 0)
    hipLaunchKernelGGL((step_kernel<T, 0>), dim3(grid_for(total)), dim3(256), 0, st, a, X, W,
                       code);
  else
    hipLaunchKernelGGL((step_kernel<T, 1>), dim3(grid_for(total)), dim3(256), 0, st, a, X, W,
                       code);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_block_step(const BlockStepArgs& a, const T* X, T* W, uint16_t* code,
                             const uint8_t* d_block_cfg, const double* d_wq, int mode,
                             hipStream_t st)
{
  if (a.lat.total == 0 || a.pieces == 0) return hipSuccess;
  const uint64_t units = (uint64_t)a.nb[0] * a.nb[1] * a.nb[2] * a.nb[3] * a.pieces;
  const unsigned grid = (unsigned)(units < (1u << 20) ? units : (1u << 20));
  if (mode == 0)
    hipLaunchKernelGGL((block_step_kernel<T, 0>), dim3(grid), dim3(256), 0, st, a, X, W, code,
                       d_block_cfg, d_wq);
  else
    hipLaunchKernelGGL((block_step_kernel<T, 1>), dim3(grid), dim3(256), 0, st, a, X, W, code,
                       d_block_cfg, d_wq);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_anchors(const Geom& g, const Lattice& lat, const T* X, T* W, uint16_t* code,
                          T* out_anchor, uint32_t R, int mode, hipStream_t st)
{
  if (lat.total == 0) return hipSuccess;
  if (mode == 0)
    hipLaunchKernelGGL((anchor_kernel<T, 0>), dim3(grid_for(lat.total)), dim3(256), 0, st, g, lat,
                       X, W, code, out_anchor, R);
  else
    hipLaunchKernelGGL((anchor_kernel<T, 1>), dim3(grid_for(lat.total)), dim3(256), 0, st, g, lat,
                       X, W, code, out_anchor, R);
  return hipGetLastError();
}

// min / max with a non-finite flag (value-range bound, Sec. 7.1.3)
// value range (exact: min and max round nothing) and the non-finite check,
// 16-byte loads, four in flight per lane; min/max in T, widened at the end
template <typename T>
__device__ __forceinline__ bool nonfinite(T v)
{
  return !(v - v == (T)0);  // inf - inf and nan - nan are nan
}

template <typename T>
__global__ void __launch_bounds__(256) minmax_kernel(const T* __restrict__ X, uint64_t n,
                                                     double* __restrict__ part, int* __restrict__ bad)
{
  __shared__ double smn[256], smx[256];
  constexpr int V = 16 / sizeof(T);  // values per 16-byte load
  if (n == 0) return;
  T mn = X[0], mx = X[0];
  bool nf = false;
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nthr = (uint64_t)gridDim.x * blockDim.x;
  const bool aligned = ((uintptr_t)X & 15) == 0;
  const uint64_t nv = aligned ? n / V : 0;  // whole vectors
  const uint4* Xv = reinterpret_cast<const uint4*>(X);
  uint64_t i = tid;
  for (; i + 3 * nthr < nv; i += 4 * nthr) {
    uint4 r[4];
#pragma unroll
    for (int u = 0; u < 4; u++) r[u] = Xv[i + u * nthr];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const T* t = reinterpret_cast<const T*>(&r[u]);
#pragma unroll
      for (int j = 0; j < V; j++) {
        nf |= nonfinite(t[j]);
        mn = t[j] < mn ? t[j] : mn;
        mx = t[j] > mx ? t[j] : mx;
      }
    }
  }
  for (; i < nv; i += nthr) {
    const uint4 r = Xv[i];
    const T* t = reinterpret_cast<const T*>(&r);
#pragma unroll
    for (int j = 0; j < V; j++) {
      nf |= nonfinite(t[j]);
      mn = t[j] < mn ? t[j] : mn;
      mx = t[j] > mx ? t[j] : mx;
    }
  }
  for (uint64_t k = nv * V + tid; k < n; k += nthr) {
    const T v = X[k];
    nf |= nonfinite(v);
    mn = v < mn ? v : mn;
    mx = v > mx ? v : mx;
  }
  if (nf) atomicOr(bad, 1);
  smn[threadIdx.x] = (double)mn;
  smx[threadIdx.x] = (double)mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      smn[threadIdx.x] = fmin(smn[threadIdx.x], smn[threadIdx.x + w]);
      smx[threadIdx.x] = fmax(smx[threadIdx.x], smx[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = smn[0];
    part[2 * blockIdx.x + 1] = smx[0];
  }
}

__global__ void __launch_bounds__(256) minmax_final_kernel(const double* __restrict__ part, int nb,
                                                           double* __restrict__ out)
{
  __shared__ double smn[256], smx[256];
  double mn = INFINITY, mx = -INFINITY;
  for (int i = threadIdx.x; i < nb; i += 256) {
    mn = fmin(mn, part[2 * i]);
    mx = fmax(mx, part[2 * i + 1]);
  }
  smn[threadIdx.x] = mn;
  smx[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      smn[threadIdx.x] = fmin(smn[threadIdx.x], smn[threadIdx.x + w]);
      smx[threadIdx.x] = fmax(smx[threadIdx.x], smx[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = smn[0];
    out[1] = smx[0];
  }
}

template <typename T>
hipError_t launch_minmax(const T* X, uint64_t n, double* d_part, int* d_bad, int nblocks,
                         hipStream_t st)
{
  hipLaunchKernelGGL((minmax_kernel<T>), dim3(nblocks), dim3(256), 0, st, X, n, d_part, d_bad);
  return hipGetLastError();
}

hipError_t launch_minmax_final(double* d_part, int nblocks, double* d_out, hipStream_t st)
{
  hipLaunchKernelGGL(minmax_final_kernel, dim3(1), dim3(256), 0, st, d_part, nblocks, d_out);
  return hipGetLastError();
}

#define INST(T)                                                                                 \
  template hipError_t launch_step<T>(const StepArgs&, const T*, T*, uint16_t*, int, hipStream_t); \
  template hipError_t launch_block_step<T>(const BlockStepArgs&, const T*, T*, uint16_t*,         \
                                           const uint8_t*, const double*, int, hipStream_t);     \
  template hipError_t launch_anchors<T>(const Geom&, const Lattice&, const T*, T*, uint16_t*, T*, \
                                        uint32_t, int, hipStream_t);                              \
  template hipError_t launch_minmax<T>(const T*, uint64_t, double*, int*, int, hipStream_t);
INST(float)
INST(double)

}  // namespace hpez
