// box_dev.h -- the level schedule of one box held in LDS (up to three dims,
// dim 2 fastest), shared by the per-block interior kernel and the tuner's
// trial kernels.  Sec. 5: every level runs its passes (1D style along the
// tuned dimension order, each optionally split in two halves for same-level
// cubic) or its multi-dimensional sub-steps; a point is predicted from box
// cells finished in earlier steps, so the box is updated in place: a cell holds
// its original value until its point is predicted, then the reconstruction.
//
// The stencils are evaluated without divergent branches: every candidate
// expression of the boundary ladder is computed from clamped (always valid)
// cells and the applicable one is selected, which is bit-identical to
// evaluating only the selected expression.
#pragma once

#include "interp_dev.h"

namespace hpez {

struct Box {
  int32_t E0, E1, E2;     // extents: neighbours are usable in [0, E - 1]
  int32_t b0, b1;         // LDS strides of dims 0 and 1 (dim 2 stride 1)
  int32_t lo0, lo1, lo2;  // first coordinate that is ever predicted
  int32_t hi0, hi1, hi2;  // last coordinate that is ever predicted
  int32_t a0, a1, a2;     // active dims
};

// smallest c >= lo with (o + c) == r (mod m), m a power of two
__device__ __forceinline__ int32_t first_in(int64_t o, int32_t lo, int32_t r, int32_t m)
{
  const int32_t x0 = (int32_t)(o & (int64_t)(m - 1)) + lo;
  return lo + ((r - x0) & (m - 1));
}

// One-dimensional prediction of the cell li at coordinate x along a dim with
// LDS stride sd (already multiplied by s); neighbours exist in [0, last].
// KIND 0 linear (Eq. 2), 1 not-a-knot (Eq. 6), 2 natural (Eq. 8); SL selects
// the same-level stencils of Eq. (13)/(14).  Near the box end the Lagrange
// polynomial through the neighbours that exist is used.
template <typename T, int KIND, int SL>
__device__ __forceinline__ T stencil_box(const T* L, int32_t li, int32_t sd, int32_t x, int32_t s,
                                         int32_t last)
{
  const bool hc = x + s <= last;
  const bool ha = x >= 3 * s;
  const T b = L[li - sd];
  const T c = L[hc ? li + sd : li - sd];
  const T a = L[ha ? li - 3 * sd : li - sd];
  const T lin = (b + c) * (T)0.5;
  const T ext = (b * (T)3 - a) * (T)0.5;
  if (KIND == 0) return hc ? lin : (ha ? ext : b);
  const bool hd = x + 3 * s <= last;
  const T d = L[hd ? li + 3 * sd : li - sd];
  T cub;
  if (KIND == 1) cub = ((b + c) * (T)9 - (a + d)) * (T)0.0625;
  else cub = ((b + c) * (T)23 - (a + d) * (T)3) * SplineK<T>::k40();
  const T qr = (b * (T)3 + c * (T)6 - d) * (T)0.125;
  const T ql = (b * (T)6 + c * (T)3 - a) * (T)0.125;
  T r = (ha && hc && hd) ? cub : (hc && hd) ? qr : (ha && hc) ? ql : hc ? lin : (ha ? ext : b);
  if (SL) {
    const bool ha2 = x >= 2 * s;
    const bool hd2 = x + 2 * s <= last;
    const T a2 = L[ha2 ? li - 2 * sd : li - sd];
    const T d2 = L[hd2 ? li + 2 * sd : li - sd];
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

// One step: every cell with c_d == r_d (mod m_d), c_d in [lo_d, hi_d], for the
// three dims.  pd >= 0: 1D prediction along pd; pd < 0: multi-dimensional over
// the odd set `odd` with weights w0..w2 (sum left to right, Eq. 12); with
// colour >= 0 only the points of that checkerboard colour (the parity of
// sum (x_d - s) / 2s over the odd dims, global coordinates x = o + c), SL
// then giving the stencil of that half (Sec. 5.4.2 carried over to MD).  NT is
// the work-group size.  The points of a step are independent, so each lane takes
// kU of them at once: op.fetch(x0, x1, x2) for all of them first (global loads
// in flight together), then the predictions and op.apply(li, x0, x1, x2, p, f).
constexpr int kU = 4;

template <typename T, int KIND, int SL, bool MD, int NT, class Op>
__device__ __forceinline__ void box_step(const Box& bx, const T* L, int32_t r0, int32_t r1,
                                         int32_t r2, int32_t m0, int32_t m1, int32_t m2,
                                         int64_t o0, int64_t o1, int64_t o2, int pd, unsigned odd,
                                         int32_t s, T w0, T w1, T w2, Op& op, int colour)
{
  const int lg2s = 31 - __clz(2 * s);
  const int32_t f0 = first_in(o0, bx.lo0, r0, m0), f1 = first_in(o1, bx.lo1, r1, m1),
                f2 = first_in(o2, bx.lo2, r2, m2);
  const int32_t c0 = f0 <= bx.hi0 ? ((bx.hi0 - f0) >> (31 - __clz(m0))) + 1 : 0;
  const int32_t c1 = f1 <= bx.hi1 ? ((bx.hi1 - f1) >> (31 - __clz(m1))) + 1 : 0;
  const int32_t c2 = f2 <= bx.hi2 ? ((bx.hi2 - f2) >> (31 - __clz(m2))) + 1 : 0;
  const uint32_t c12 = (uint32_t)(c1 * c2);
  const uint32_t total = (uint32_t)c0 * c12;
  // waves with no point in this step skip it before any further setup
  if ((threadIdx.x & ~63u) >= total) return;
  const Divisor mg12 = fmagic(c12);
  const Divisor mg2 = fmagic((uint32_t)c2);
  // plain values first: a select between two fields of bx would keep bx in memory
  const int32_t B0 = bx.b0, B1 = bx.b1, L0 = bx.E0 - 1, L1 = bx.E1 - 1, L2 = bx.E2 - 1;
  const int32_t bsd = pd == 0 ? B0 : (pd == 1 ? B1 : 1);
  const int32_t last = pd == 0 ? L0 : (pd == 1 ? L1 : L2);
  const int32_t sd = s * bsd;
  for (uint32_t kb = 0; kb < total; kb += kU * NT) {
    int32_t x0[kU], x1[kU], x2[kU];
    typename Op::Fetched fv[kU];
#pragma unroll
    for (int u = 0; u < kU; u++) {
      const uint32_t k = kb + u * NT + threadIdx.x;
      const uint32_t kk = k < total ? k : 0u;
      const uint32_t i0 = fdiv(kk, mg12);
      const uint32_t rem = kk - i0 * c12;
      const uint32_t i1 = fdiv(rem, mg2);
      const uint32_t i2 = rem - i1 * (uint32_t)c2;
      x0[u] = f0 + (int32_t)i0 * m0;
      x1[u] = f1 + (int32_t)i1 * m1;
      x2[u] = f2 + (int32_t)i2 * m2;
      fv[u] = op.fetch(x0[u], x1[u], x2[u], k < total);
    }
#pragma unroll
    for (int u = 0; u < kU; u++) {
      if (kb + u * NT + threadIdx.x >= total) continue;
      if (MD && colour >= 0) {
        const int64_t c = ((odd & 1u) ? ((o0 + x0[u]) >> lg2s) : 0) +
                          ((odd & 2u) ? ((o1 + x1[u]) >> lg2s) : 0) +
                          ((odd & 4u) ? ((o2 + x2[u]) >> lg2s) : 0);
        if ((int)(c & 1) != colour) continue;
      }
      const int32_t li = x0[u] * B0 + x1[u] * B1 + x2[u];
      T p;
      if (!MD) {
        const int32_t xd = pd == 0 ? x0[u] : (pd == 1 ? x1[u] : x2[u]);
        p = stencil_box<T, KIND, SL>(L, li, sd, xd, s, last);
      } else {
        bool first = true;
        T acc = (T)0;
        if (odd & 1u) {
          acc = w0 * stencil_box<T, KIND, SL>(L, li, s * B0, x0[u], s, L0);
          first = false;
        }
        if (odd & 2u) {
          const T t = w1 * stencil_box<T, KIND, SL>(L, li, s * B1, x1[u], s, L1);
          acc = first ? t : acc + t;
          first = false;
        }
        if (odd & 4u) {
          const T t = w2 * stencil_box<T, KIND, SL>(L, li, s, x2[u], s, L2);
          acc = first ? t : acc + t;
        }
        p = acc;
      }
      op.apply(li, x0[u], x1[u], x2[u], p, fv[u]);
    }
  }
}

template <typename T, int KIND, int SL, int NT, class Op>
__device__ __forceinline__ void box_step_k(bool md, const Box& bx, const T* L, int32_t r0, int32_t r1,
                                           int32_t r2, int32_t m0, int32_t m1, int32_t m2, int64_t o0,
                                           int64_t o1, int64_t o2, int pd, unsigned odd, int32_t s,
                                           T w0, T w1, T w2, Op& op, int colour)
{
  if (md)
    box_step<T, KIND, SL, true, NT>(bx, L, r0, r1, r2, m0, m1, m2, o0, o1, o2, pd, odd, s, w0, w1,
                                    w2, op, colour);
  else
    box_step<T, KIND, SL, false, NT>(bx, L, r0, r1, r2, m0, m1, m2, o0, o1, o2, pd, odd, s, w0, w1,
                                     w2, op, -1);
}

// runtime (uniform) kind / same-level / paradigm to the compiled step
template <typename T, int NT, class Op>
__device__ __forceinline__ void box_step_any(int kind, int sl, bool md, const Box& bx, const T* L,
                                             int32_t r0, int32_t r1, int32_t r2, int32_t m0,
                                             int32_t m1, int32_t m2, int64_t o0, int64_t o1,
                                             int64_t o2, int pd, unsigned odd, int32_t s, T w0, T w1,
                                             T w2, Op& op, int colour = -1)
{
  if (kind == 0)
    box_step_k<T, 0, 0, NT>(md, bx, L, r0, r1, r2, m0, m1, m2, o0, o1, o2, pd, odd, s, w0, w1, w2, op,
                            colour);
  else if (kind == 1 && sl)
    box_step_k<T, 1, 1, NT>(md, bx, L, r0, r1, r2, m0, m1, m2, o0, o1, o2, pd, odd, s, w0, w1, w2, op,
                            colour);
  else if (kind == 1)
    box_step_k<T, 1, 0, NT>(md, bx, L, r0, r1, r2, m0, m1, m2, o0, o1, o2, pd, odd, s, w0, w1, w2, op,
                            colour);
  else if (sl)
    box_step_k<T, 2, 1, NT>(md, bx, L, r0, r1, r2, m0, m1, m2, o0, o1, o2, pd, odd, s, w0, w1, w2, op,
                            colour);
  else
    box_step_k<T, 2, 0, NT>(md, bx, L, r0, r1, r2, m0, m1, m2, o0, o1, o2, pd, odd, s, w0, w1, w2, op,
                            colour);
}

// One level (stride s) with configuration c: all its steps, each followed by a
// work-group barrier.  The box origin (o0, o1, o2) fixes the residues (the
// lattice is global: coordinates o + c).  wmd: MD weights [kind][odd set < 8][dim < 4].
template <typename T, int NT, class Op>
__device__ __forceinline__ void box_level(const hpez_interp& c, const Box& bx, T* L, int64_t o0,
                                          int64_t o1, int64_t o2, int32_t s, const double* wmd,
                                          Op& op)
{
  const int a0 = bx.a0, a1 = bx.a1, a2 = bx.a2;
  if (c.md) {
    // with same-level cubic each sub-step runs in two halves by checkerboard
    // colour, the second with the same-level stencils
    const int nact = a0 + a1 + a2;
    const int32_t m0 = a0 ? 2 * s : 1, m1 = a1 ? 2 * s : 1, m2 = a2 ? 2 * s : 1;
    const bool halves = c.kind != 0 && c.same_level;
    for (int cnt = 1; cnt <= nact; cnt++) {
      for (int half = 0; half < (halves ? 2 : 1); half++) {
        for (unsigned odd = 1; odd < 8; odd++) {
          if ((int)__popc(odd) != cnt) continue;
          if (((odd & 1u) && !a0) || ((odd & 2u) && !a1) || ((odd & 4u) && !a2)) continue;
          const int32_t r0 = (odd & 1u) ? s : 0, r1 = (odd & 2u) ? s : 0, r2 = (odd & 4u) ? s : 0;
          const double* w = wmd + (c.kind * 8 + odd) * 4;
          box_step_any<T, NT>(c.kind, half, true, bx, L, r0, r1, r2, m0, m1, m2, o0, o1, o2, -1, odd,
                              s, (T)w[0], (T)w[1], (T)w[2], op, halves ? half : -1);
        }
        __syncthreads();
      }
    }
    return;
  }
  // pass order over the active dims, two bits per pass
  const unsigned actm = (unsigned)a0 | (unsigned)a1 << 1 | (unsigned)a2 << 2;
  unsigned seen = 0, pds = 0;
  int np = 0;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const unsigned d = (unsigned)c.order[i];
    if (d < 3 && (actm >> d & 1u) && !(seen >> d & 1u)) {
      seen |= 1u << d;
      pds |= d << (2 * np);
      np++;
    }
  }
  const bool halves = c.kind != 0 && c.same_level;
  unsigned earlier = 0;  // dims of earlier passes: multiples of s; later: of 2s
  for (int k = 0; k < np; k++) {
    const int pd = (int)(pds >> (2 * k) & 3u);
    int32_t r0 = 0, r1 = 0, r2 = 0;
    int32_t m0 = !a0 ? 1 : ((earlier & 1u) ? s : 2 * s);
    int32_t m1 = !a1 ? 1 : ((earlier & 2u) ? s : 2 * s);
    int32_t m2 = !a2 ? 1 : ((earlier & 4u) ? s : 2 * s);
    for (int half = 0; half < (halves ? 2 : 1); half++) {
      const int32_t rh = half ? 3 * s : s;
      const int32_t mh = halves ? 4 * s : 2 * s;
      if (pd == 0) { r0 = rh; m0 = mh; }
      if (pd == 1) { r1 = rh; m1 = mh; }
      if (pd == 2) { r2 = rh; m2 = mh; }
      box_step_any<T, NT>(c.kind, half, false, bx, L, r0, r1, r2, m0, m1, m2, o0, o1, o2, pd, 0u, s,
                          (T)0, (T)0, (T)0, op);
      __syncthreads();
    }
    earlier |= 1u << pd;
  }
}

}  // namespace hpez
