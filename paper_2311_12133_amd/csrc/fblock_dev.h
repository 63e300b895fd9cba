// fblock_dev.h -- the levels below the block's coarse lattice (strides 2 and 1)
// of a full block: a 32^3 brick with all three dims active and a box of 32 or
// 33 cells per dim (the far face is absent at the grid end).  Same schedule,
// stencils and quantizer as box_level (Sec. 5.2-5.4, Eq. 2/6/8/13/14, the
// multi-dimensional weights of Eq. 12), on a box layout chosen for the
// schedule:
//
//   * every dim's coordinates are split by parity: coordinate c sits at slot
//     c / 2 when even (0..16) and 17 + c / 2 when odd (17..32).  At the two
//     finest levels a step's points then fill whole slot ranges along each dim
//     (contiguous at stride 1, every other slot at stride 2), and a stencil's
//     neighbours along a dim sit at fixed slot offsets from the point;
//   * lanes map to a step's points by power-of-two padded ranges: the dim-2
//     and dim-1 indices are fixed per lane, only the dim-0 index advances, so
//     a point costs one address increment instead of a division.
#pragma once

#include "block_dev.h"
#include "interp_dev.h"

namespace hpez {

constexpr int32_t kFP1 = 33;            // slot pitch of dim 1
constexpr int32_t kFP0 = 33 * 33;       // slot pitch of dim 0

__device__ __forceinline__ int32_t fslot(int32_t c) { return (c & 1) ? 17 + (c >> 1) : (c >> 1); }
__device__ __forceinline__ int32_t fcoord(int32_t sl) { return sl <= 16 ? 2 * sl : 2 * sl - 33; }

// Point classes of a dim in one step at stride s: EVEN multiples of 2s, ODD
// (s mod 2s), ANY multiples of s, H1 (s mod 4s) and H3 (3s mod 4s), all within
// the interior coordinates 1..31 (0 and 32 are block faces).
enum FCls { kEven = 0, kOdd = 1, kAny = 2, kH1 = 3, kH3 = 4 };

// slots f + i t for i < n, padded to 2^l; `gap`: level 1 ANY, whose index 15
// (slot 16, the far face) is skipped
struct FRange {
  int32_t f, t, n, l;
  bool gap;
};

__device__ __forceinline__ FRange frange(int cls, int s)
{
  if (s == 1) {
    switch (cls) {
      case kEven: return {1, 1, 15, 4, false};
      case kOdd: return {17, 1, 16, 4, false};
      case kAny: return {1, 1, 32, 5, true};
      case kH1: return {17, 2, 8, 3, false};
      default: return {18, 2, 8, 3, false};
    }
  }
  switch (cls) {  // s == 2
    case kEven: return {2, 2, 7, 3, false};
    case kOdd: return {1, 2, 8, 3, false};
    case kAny: return {1, 1, 15, 4, false};
    case kH1: return {1, 4, 4, 2, false};
    default: return {3, 4, 4, 2, false};
  }
}

// Neighbour slot offsets of a point of stride s along a dim (b = x - s,
// c = x + s, a = x - 3s, d = x + 3s, a2 = x - 2s, d2 = x + 2s).
struct FOff {
  int32_t b, c, a, d, a2, d2;
};
__device__ __forceinline__ FOff foff(int s, int32_t pitch)
{
  if (s == 1) return {-17 * pitch, -16 * pitch, -18 * pitch, -15 * pitch, -pitch, pitch};
  return {-pitch, pitch, -3 * pitch, 3 * pitch, -2 * pitch, 2 * pitch};
}

// The stencil of box_dev.h's stencil_box with the neighbours at offsets o from
// cell li: the boundary ladder's candidates are computed from clamped cells
// and the applicable one selected.
template <typename T, int KIND, int SL>
__device__ __forceinline__ T fstencil(const T* L, int32_t li, const FOff& o, int32_t x, int32_t s,
                                      int32_t last)
{
  const bool hc = x + s <= last;
  const bool ha = x >= 3 * s;
  const T b = L[li + o.b];
  const T c = L[li + (hc ? o.c : o.b)];
  const T a = L[li + (ha ? o.a : o.b)];
  const T lin = (b + c) * (T)0.5;
  const T ext = (b * (T)3 - a) * (T)0.5;
  if (KIND == 0) return hc ? lin : (ha ? ext : b);
  const bool hd = x + 3 * s <= last;
  const T d = L[li + (hd ? o.d : o.b)];
  T cub;
  if (KIND == 1) cub = ((b + c) * (T)9 - (a + d)) * (T)0.0625;
  else cub = ((b + c) * (T)23 - (a + d) * (T)3) * SplineK<T>::k40();
  const T qr = (b * (T)3 + c * (T)6 - d) * (T)0.125;
  const T ql = (b * (T)6 + c * (T)3 - a) * (T)0.125;
  T r = (ha && hc && hd) ? cub : (hc && hd) ? qr : (ha && hc) ? ql : hc ? lin : (ha ? ext : b);
  if (SL) {
    const bool ha2 = x >= 2 * s;
    const bool hd2 = x + 2 * s <= last;
    const T a2 = L[li + (ha2 ? o.a2 : o.b)];
    const T d2 = L[li + (hd2 ? o.d2 : o.b)];
    if (KIND == 1) {
      const T v = ((b + c) * (T)4 - (a2 + d2)) * SplineK<T>::k6();
      r = (ha2 && hc && hd2) ? v : r;
    } else {
      const T v = ((b + c) * (T)46 - (a2 + d2) * (T)18 + (a + d) * (T)3) * SplineK<T>::k62();
      r = (ha && ha2 && hc && hd2 && hd) ? v : r;
    }
  }
  return r;
}

// Per-block state of the full-block schedule.  MODE 0 compresses (codes to
// the brick, histogram), MODE 1 reconstructs (codes from the brick).
template <typename T>
struct FBlock {
  T* L;
  HPEZ_GLOBAL uint16_t* code;         // the brick's 32^3 codes (row-major)
  const HPEZ_GLOBAL T* out;           // decompress: the field (verbatim values at code 0)
  uint32_t* lh;                       // LDS histogram window
  HPEZ_GLOBAL uint32_t* hist;
  int64_t o0, o1, o2, st0, st1;       // brick origin and field strides
  int32_t last0, last1, last2;        // last box coordinate per dim (31 or 32)
  uint32_t R, lo;
  double el, inv2e, twoe;
  uint32_t nR;
};

// Linear stencil of an interior point (x + s <= last along its dim, so the
// first rung of the ladder applies): Eq. (2).
template <typename T>
__device__ __forceinline__ T flin(const T* L, int32_t li, const FOff& o)
{
  return (L[li + o.b] + L[li + o.c]) * (T)0.5;
}

// One step: the points whose dim-d coordinate is of class cls_d at stride S;
// pd >= 0 a 1D pass along pd, else multi-dimensional over the odd set `odd`
// with weights w0..w2 summed left to right (ascending dims).  INNER: every
// stencil dim of the step has its far face in the box (last = 32), so every
// point has its c neighbour.  Decompressing, each cell of an interior point
// holds its code (loaded with the box) until the point is reconstructed.
template <typename T, int KIND, int SL, bool MD, int MODE, int NT, bool INNER, int S>
__device__ __forceinline__ void fstep(FBlock<T>& fb, int cls0, int cls1, int cls2, int pd,
                                      unsigned odd, T w0, T w1, T w2)
{
  const FRange r0 = frange(cls0, S), r1 = frange(cls1, S), r2 = frange(cls2, S);
  const int32_t l12 = r1.l + r2.l;
  const int32_t t = (int32_t)threadIdx.x;
  const int32_t i2 = t & ((1 << r2.l) - 1);
  const int32_t i1 = (t >> r2.l) & ((1 << r1.l) - 1);
  const int32_t n0 = r0.gap ? 32 : r0.n;
  int32_t i0 = t >> l12;
  // waves whose first lane is past the step skip it
  if (((t & ~63) >> l12) >= n0) return;
  const bool ok12 = i1 < (r1.gap ? 32 : r1.n) && i2 < (r2.gap ? 32 : r2.n) &&
                    !(r1.gap && i1 == 15) && !(r2.gap && i2 == 15);
  if (!ok12) return;
  const int32_t di0 = NT >> l12;
  const int32_t s1 = r1.f + i1 * r1.t, s2 = r2.f + i2 * r2.t;
  const int32_t c1 = fcoord(s1), c2 = fcoord(s2);
  const int32_t base12 = s1 * kFP1 + s2;
  const int32_t cb12 = c1 * 32 + c2;
  // plain values (a select between fields of fb would keep fb in memory)
  const int32_t last0 = fb.last0, last1 = fb.last1, last2 = fb.last2;
  const FOff f0 = foff(S, kFP0), f1 = foff(S, kFP1), f2 = foff(S, 1);
  const FOff fp = pd == 0 ? f0 : (pd == 1 ? f1 : f2);
  const int32_t lastp = pd == 0 ? last0 : (pd == 1 ? last1 : last2);
  const int32_t r0f = r0.f, r0t = r0.t;
  const bool gap0 = r0.gap;
  T* L = fb.L;
  const uint32_t R = fb.R, lo = fb.lo;
  const double el = fb.el, inv2e = fb.inv2e, twoe = fb.twoe;
  uint32_t nR = 0;
  // one point per round: the registers of more points in flight cost more
  // than their overlapped LDS latency gains (a work-group fills the CU)
  for (; i0 < n0; i0 += di0) {
    if (gap0 && i0 == 15) continue;
    const int32_t s0 = r0f + i0 * r0t;
    const int32_t li = s0 * kFP0 + base12;
    const int32_t c0 = fcoord(s0);
    T p;
    if (!MD) {
      const int32_t xd = pd == 0 ? c0 : (pd == 1 ? c1 : c2);
      p = (INNER && KIND == 0) ? flin<T>(L, li, fp) : fstencil<T, KIND, SL>(L, li, fp, xd, S, lastp);
    } else {
      bool first = true;
      T acc = (T)0;
      if (odd & 1u) {
        acc = w0 * ((INNER && KIND == 0) ? flin<T>(L, li, f0)
                                         : fstencil<T, KIND, 0>(L, li, f0, c0, S, last0));
        first = false;
      }
      if (odd & 2u) {
        const T v = w1 * ((INNER && KIND == 0) ? flin<T>(L, li, f1)
                                               : fstencil<T, KIND, 0>(L, li, f1, c1, S, last1));
        acc = first ? v : acc + v;
        first = false;
      }
      if (odd & 4u) {
        const T v = w2 * ((INNER && KIND == 0) ? flin<T>(L, li, f2)
                                               : fstencil<T, KIND, 0>(L, li, f2, c2, S, last2));
        acc = first ? v : acc + v;
      }
      p = acc;
    }
    if (MODE == 0) {
      const T xv = L[li];
      T xr = xv;
      const uint32_t q = quantize<T>(xv, p, inv2e, twoe, el, R, xr);
      fb.code[(uint32_t)(c0 * 1024 + cb12)] = (uint16_t)q;
      L[li] = xr;
      nR += q == R;
      if (q != R) {
        const uint32_t w = q - lo;
        if (w < (uint32_t)kBlockHistWin)
          __hip_atomic_fetch_add(&fb.lh[w], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else
          __hip_atomic_fetch_add(&fb.hist[q], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    } else {
      static_assert(MODE == 0 || sizeof(T) == 4, "codes held in float cells");
      const uint32_t q = __float_as_uint((float)L[li]);
      L[li] = q ? recon<T>(p, (double)((int32_t)q - (int32_t)R), twoe)
                : fb.out[(fb.o0 + c0) * fb.st0 + (fb.o1 + c1) * fb.st1 + (fb.o2 + c2)];
    }
  }
  fb.nR += nR;
}

// runtime kind / same-level / paradigm to the compiled step; linear steps whose
// stencil dims all reach their far face take the interior form
template <typename T, int MODE, int NT, int S>
__device__ __forceinline__ void fstep_any(FBlock<T>& fb, int kind, int sl, bool md, int c0, int c1,
                                          int c2, int pd, unsigned odd, T w0, T w1, T w2)
{
  const unsigned dims = md ? odd : (1u << pd);
  const bool inner = (!(dims & 1u) || fb.last0 == 32) && (!(dims & 2u) || fb.last1 == 32) &&
                     (!(dims & 4u) || fb.last2 == 32);
  if (md) {
    if (kind == 0 && inner) fstep<T, 0, 0, true, MODE, NT, true, S>(fb, c0, c1, c2, -1, odd, w0, w1, w2);
    else if (kind == 0) fstep<T, 0, 0, true, MODE, NT, false, S>(fb, c0, c1, c2, -1, odd, w0, w1, w2);
    else if (kind == 1) fstep<T, 1, 0, true, MODE, NT, false, S>(fb, c0, c1, c2, -1, odd, w0, w1, w2);
    else fstep<T, 2, 0, true, MODE, NT, false, S>(fb, c0, c1, c2, -1, odd, w0, w1, w2);
    return;
  }
  if (kind == 0 && inner) fstep<T, 0, 0, false, MODE, NT, true, S>(fb, c0, c1, c2, pd, 0u, w0, w1, w2);
  else if (kind == 0) fstep<T, 0, 0, false, MODE, NT, false, S>(fb, c0, c1, c2, pd, 0u, w0, w1, w2);
  else if (kind == 1 && sl) fstep<T, 1, 1, false, MODE, NT, false, S>(fb, c0, c1, c2, pd, 0u, w0, w1, w2);
  else if (kind == 1) fstep<T, 1, 0, false, MODE, NT, false, S>(fb, c0, c1, c2, pd, 0u, w0, w1, w2);
  else if (sl) fstep<T, 2, 1, false, MODE, NT, false, S>(fb, c0, c1, c2, pd, 0u, w0, w1, w2);
  else fstep<T, 2, 0, false, MODE, NT, false, S>(fb, c0, c1, c2, pd, 0u, w0, w1, w2);
}

// One level (stride S = 2 or 1) of a full block with configuration c, each
// step followed by a work-group barrier (as box_level).
template <typename T, int MODE, int NT, int S>
__device__ __forceinline__ void flevel(const hpez_interp& c, FBlock<T>& fb, const double* wmd)
{
  if (c.md) {
    for (int cnt = 1; cnt <= 3; cnt++) {
      for (unsigned odd = 1; odd < 8; odd++) {
        if ((int)__popc(odd) != cnt) continue;
        const double* w = wmd + (c.kind * 8 + odd) * 4;
        fstep_any<T, MODE, NT, S>(fb, c.kind, 0, true, (odd & 1u) ? kOdd : kEven,
                               (odd & 2u) ? kOdd : kEven, (odd & 4u) ? kOdd : kEven, -1, odd,
                               (T)w[0], (T)w[1], (T)w[2]);
      }
      __syncthreads();
    }
    return;
  }
  unsigned seen = 0, pds = 0;
  int np = 0;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const unsigned d = (unsigned)c.order[i];
    if (d < 3 && !(seen >> d & 1u)) {
      seen |= 1u << d;
      pds |= d << (2 * np);
      np++;
    }
  }
  const bool halves = c.kind != 0 && c.same_level;
  unsigned earlier = 0;
  for (int k = 0; k < np; k++) {
    const int pd = (int)(pds >> (2 * k) & 3u);
    for (int half = 0; half < (halves ? 2 : 1); half++) {
      const int pc = halves ? (half ? kH3 : kH1) : kOdd;
      const int cl0 = pd == 0 ? pc : ((earlier & 1u) ? kAny : kEven);
      const int cl1 = pd == 1 ? pc : ((earlier & 2u) ? kAny : kEven);
      const int cl2 = pd == 2 ? pc : ((earlier & 4u) ? kAny : kEven);
      fstep_any<T, MODE, NT, S>(fb, c.kind, half, false, cl0, cl1, cl2, pd, 0u, (T)0, (T)0, (T)0);
      __syncthreads();
    }
    earlier |= 1u << pd;
  }
}

}  // namespace hpez
