// k_block.hip -- block-wise interpolation on MI355X (Sec. 6.6 configurations,
// Sec. 5 predictor), for block side B = 32 (the paper's default, equal to the
// stream's brick side) and grids of up to three dimensions.
//
// With block-wise configurations, levels with stride s < B are computed in two
// phases (the reading the whole library uses for how blocks meet):
//   * faces: points with some active coordinate a multiple of B, with the
//     level's global configuration.  A face point is never interpolated along
//     the dimension that makes it a face, so every stencil stays inside its
//     face plane.  Face values and codes live in compact per-family arrays
//     (family d = the planes x_d = 0, B, 2B, ...; layout [plane][other dims],
//     so every plane is contiguous);
//   * interiors: one work-group per block runs every level s < B for the
//     block's own configuration, stencils clipped to the block's closed box.
//     The box (B+1)^D lives in LDS and is updated in place: a cell holds the
//     original value until its point is predicted, then the reconstruction.
//     The work-group then writes the block's whole brick of codes (near-face
//     codes copied from the face arrays) and histograms it.

#include "block_dev.h"
#include "interp_dev.h"

namespace hpez {

__device__ __forceinline__ int64_t face_index(const FaceGeo& f, int e, const int64_t* x)
{
  int64_t i = (x[e] >> f.blog2) * f.plane[e];
  for (int k = 0; k < 4; k++)
    if (k != e) i += x[k] * f.fs[e][k];
  return i;
}

// write a face point's value (and code) into every family it belongs to
template <typename T>
__device__ __forceinline__ void face_store(const FaceGeo& f, const Geom& g, const int64_t* x, T v,
                                           uint16_t q, bool with_code)
{
  for (int e = 0; e < 4; e++) {
    if (!g.act[e] || (x[e] & (f.B - 1))) continue;
    const int64_t fi = face_index(f, e, x);
    reinterpret_cast<T*>(f.val[e])[fi] = v;
    if (with_code) f.code[e][fi] = q;
  }
}

// ---------------------------------------------------------------------------
// points on the coarse grid of stride B (anchors and levels s >= B): copy the
// working grid and codes into the face arrays
template <typename T, int MODE>
__global__ void __launch_bounds__(256) face_init_kernel(FaceGeo f, Geom g, Lattice lat,
                                                        const T* __restrict__ W,
                                                        const uint16_t* __restrict__ code)
{
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < lat.total; k += stride) {
    int64_t x[4];
    lattice_point(lat, k, x);
    const int64_t idx = x[0] * g.st[0] + x[1] * g.st[1] + x[2] * g.st[2] + x[3];
    const uint16_t q = MODE == 0 ? code[brick_pos(g.n, x)] : (uint16_t)0;
    face_store<T>(f, g, x, W[idx], q, MODE == 0);
  }
}

// one step of the face phase for one family
template <typename T, int MODE>
__global__ void __launch_bounds__(256) face_step_kernel(FaceStep a, FaceGeo f,
                                                        const T* __restrict__ X,
                                                        uint16_t* __restrict__ code,
                                                        const T* __restrict__ out)
{
  const int d = a.fam;
  const T* __restrict__ F = reinterpret_cast<const T*>(f.val[d]);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < a.total; k += stride) {
    // plane index slowest, other dims row-major (last dim fastest)
    int64_t x[4];
    uint64_t r = k;
    for (int e = 3; e >= 0; e--) {
      if (e == d) continue;
      const uint64_t q = r / a.cnt[e];
      x[e] = a.first[e] + (int64_t)(r - q * a.cnt[e]) * a.step[e];
      r = q;
    }
    x[d] = (int64_t)r * f.B;
    bool skip = false;
    for (int e = 0; e < d; e++)
      if (a.g.act[e] && (x[e] & (f.B - 1)) == 0) skip = true;  // belongs to family e
    if (skip) continue;
    const int64_t fi = face_index(f, d, x);
    T p;
    if (!a.md) {
      const int e = a.pdim;
      p = spline<T, T>(F, fi, a.s * f.fs[d][e], x[e], a.s, 0, a.g.n[e] - 1, a.kind, a.sl);
    } else {
      bool first = true;
      T acc = (T)0;
      for (int e = 0; e < 4; e++) {
        if (!(a.odd >> e & 1u)) continue;
        const T pe = spline<T, T>(F, fi, a.s * f.fs[d][e], x[e], a.s, 0, a.g.n[e] - 1, a.kind, 0);
        const T term = (T)a.wq[e] * pe;
        acc = first ? term : acc + term;
        first = false;
      }
      p = acc;
    }
    const int64_t idx = x[0] * a.g.st[0] + x[1] * a.g.st[1] + x[2] * a.g.st[2] + x[3];
    if (MODE == 0) {
      const T xv = X[idx];
      T xr = xv;
      const uint32_t q = quantize<T>(xv, p, a.inv2e, a.twoe, a.el, a.R, xr);
      face_store<T>(f, a.g, x, q ? xr : xv, (uint16_t)q, true);
    } else {
      const uint32_t q = code[brick_pos(a.g.n, x)];
      const T v = q ? (T)((double)p + (double)((int64_t)q - (int64_t)a.R) * a.twoe) : out[idx];
      face_store<T>(f, a.g, x, v, 0, false);
    }
  }
}

// ---------------------------------------------------------------------------
// interiors: one work-group per block, the whole schedule below B in LDS.
// The grid has at most three dims here (dims 0..2; dim 3 has size 1), so all
// per-dimension quantities are scalars (no per-lane arrays, no scratch).

// exact n / d for n, d < 2^16 (so n * d < 2^32) with m = ceil(2^32 / d); for
// d = 1 the multiplier 2^32 does not fit and is stored as 0
__device__ __forceinline__ uint32_t fmagic(uint32_t d) { return (uint32_t)((0xFFFFFFFFull / d) + 1); }
__device__ __forceinline__ uint32_t fdiv(uint32_t n, uint32_t m) { return m ? __umulhi(n, m) : n; }

struct Box3 {
  int64_t o0, o1, o2;   // block origin
  int32_t E0, E1, E2;   // box extents (closed box along active dims)
  int32_t h0, h1, h2;   // last interior coordinate
  int32_t l0, l1, l2;   // first interior coordinate (1 along active dims, else 0)
  int32_t b0, b1;       // LDS strides of dims 0 and 1 (dim 2 stride 1)
  int32_t Eb0, Eb1, Eb2;  // brick extents
};

__device__ __forceinline__ void box3(const Geom& g, int64_t bi, const int64_t* nb, Box3& x)
{
  const int64_t q2 = bi / nb[2];
  const int64_t i2 = bi - q2 * nb[2];
  const int64_t i0 = q2 / nb[1];
  const int64_t i1 = q2 - i0 * nb[1];
  x.o0 = i0 * kBrick;
  x.o1 = i1 * kBrick;
  x.o2 = i2 * kBrick;
  const int64_t r0 = g.n[0] - x.o0, r1 = g.n[1] - x.o1, r2 = g.n[2] - x.o2;
  x.Eb0 = (int32_t)(r0 < kBrick ? r0 : kBrick);
  x.Eb1 = (int32_t)(r1 < kBrick ? r1 : kBrick);
  x.Eb2 = (int32_t)(r2 < kBrick ? r2 : kBrick);
  x.E0 = g.act[0] ? (int32_t)(r0 < kBrick + 1 ? r0 : kBrick + 1) : x.Eb0;
  x.E1 = g.act[1] ? (int32_t)(r1 < kBrick + 1 ? r1 : kBrick + 1) : x.Eb1;
  x.E2 = g.act[2] ? (int32_t)(r2 < kBrick + 1 ? r2 : kBrick + 1) : x.Eb2;
  x.h0 = x.Eb0 - 1;
  x.h1 = x.Eb1 - 1;
  x.h2 = x.Eb2 - 1;
  x.l0 = g.act[0] ? 1 : 0;
  x.l1 = g.act[1] ? 1 : 0;
  x.l2 = g.act[2] ? 1 : 0;
  x.b1 = x.E2;
  x.b0 = x.E1 * x.E2;
}

// smallest c >= lo with (o + c) == r (mod m), m a power of two
__device__ __forceinline__ int32_t first_in(int64_t o, int32_t lo, int32_t r, int32_t m)
{
  const int32_t x0 = (int32_t)(o & (int64_t)(m - 1)) + lo;  // o + lo modulo m, offset kept
  const int32_t d = (r - x0) & (m - 1);
  return lo + d;
}

// one step: every interior point with coordinates c_d == r_d (mod m_d) along the
// three dims; pd is the pass dim (1D style) or -1 with the odd set (MD)
template <typename T, int MODE>
__device__ __forceinline__ void interior_step(const BlockArgs& a, const Box3& bx, T* L, int32_t r0,
                                              int32_t r1, int32_t r2, int32_t m0, int32_t m1,
                                              int32_t m2, int kind, int sl, int pd, unsigned odd,
                                              int32_t s, double el, double inv2e, double twoe,
                                              const double* __restrict__ wq,
                                              uint16_t* __restrict__ code, uint64_t brick_base,
                                              const T* __restrict__ out)
{
  const int32_t f0 = first_in(bx.o0, bx.l0, r0, m0), f1 = first_in(bx.o1, bx.l1, r1, m1),
                f2 = first_in(bx.o2, bx.l2, r2, m2);
  const int32_t c0 = f0 <= bx.h0 ? (bx.h0 - f0) / m0 + 1 : 0;
  const int32_t c1 = f1 <= bx.h1 ? (bx.h1 - f1) / m1 + 1 : 0;
  const int32_t c2 = f2 <= bx.h2 ? (bx.h2 - f2) / m2 + 1 : 0;
  const uint32_t c12 = (uint32_t)(c1 * c2);
  const uint32_t total = (uint32_t)c0 * c12;
  if (!total) return;
  const uint32_t mg12 = fmagic(c12), mg2 = fmagic((uint32_t)c2);
  // stride and extent of the pass dim (uniform)
  const int32_t B0 = bx.b0, B1 = bx.b1, E0 = bx.E0, E1 = bx.E1, E2 = bx.E2;
  int32_t bsd = 1, Ed = E2;
  if (pd == 0) {
    bsd = B0;
    Ed = E0;
  } else if (pd == 1) {
    bsd = B1;
    Ed = E1;
  }
  T w0 = 0, w1 = 0, w2 = 0;
  if (pd < 0) {
    w0 = (T)wq[(kind * 16 + odd) * 4 + 0];
    w1 = (T)wq[(kind * 16 + odd) * 4 + 1];
    w2 = (T)wq[(kind * 16 + odd) * 4 + 2];
  }
  for (uint32_t k = threadIdx.x; k < total; k += blockDim.x) {
    const uint32_t i0 = fdiv(k, mg12);
    const uint32_t rem = k - i0 * c12;
    const uint32_t i1 = fdiv(rem, mg2);
    const uint32_t i2 = rem - i1 * (uint32_t)c2;
    const int32_t x0 = f0 + (int32_t)i0 * m0, x1 = f1 + (int32_t)i1 * m1, x2 = f2 + (int32_t)i2 * m2;
    const int32_t li = x0 * bx.b0 + x1 * bx.b1 + x2;
    T p;
    if (pd >= 0) {
      const int32_t xd = pd == 0 ? x0 : pd == 1 ? x1 : x2;
      p = spline<T, T>(L, li, (int64_t)s * bsd, xd, s, 0, Ed - 1, kind, sl);
    } else {
      bool first = true;
      T acc = (T)0;
      if (odd & 1u) {
        const T t = w0 * spline<T, T>(L, li, (int64_t)s * bx.b0, x0, s, 0, bx.E0 - 1, kind, 0);
        acc = t;
        first = false;
      }
      if (odd & 2u) {
        const T t = w1 * spline<T, T>(L, li, (int64_t)s * bx.b1, x1, s, 0, bx.E1 - 1, kind, 0);
        acc = first ? t : acc + t;
        first = false;
      }
      if (odd & 4u) {
        const T t = w2 * spline<T, T>(L, li, (int64_t)s, x2, s, 0, bx.E2 - 1, kind, 0);
        acc = first ? t : acc + t;
      }
      p = acc;
    }
    const uint64_t cpos = brick_base + (uint64_t)((x0 * bx.Eb1 + x1) * bx.Eb2 + x2);
    if (MODE == 0) {
      const T xv = L[li];
      T xr = xv;
      const uint32_t q = quantize<T>(xv, p, inv2e, twoe, el, a.R, xr);
      code[cpos] = (uint16_t)q;
      L[li] = q ? xr : xv;
    } else {
      const uint32_t q = code[cpos];
      if (q) {
        L[li] = (T)((double)p + (double)((int64_t)q - (int64_t)a.R) * twoe);
      } else {
        L[li] = out[(bx.o0 + x0) * a.g.st[0] + (bx.o1 + x1) * a.g.st[1] + (bx.o2 + x2)];
      }
    }
  }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(1024) block_kernel(BlockArgs a, FaceGeo f, const T* __restrict__ X,
                                                     uint16_t* __restrict__ code,
                                                     const uint8_t* __restrict__ bcfg,
                                                     const double* __restrict__ wq,
                                                     uint32_t* __restrict__ hist, T* __restrict__ out)
{
  extern __shared__ unsigned char lds_raw[];
  T* L = reinterpret_cast<T*>(lds_raw);
  const int64_t bi = blockIdx.x;
  Box3 bx;
  box3(a.g, bi, a.nb, bx);
  const int64_t st0 = a.g.st[0], st1 = a.g.st[1];
  // stream position of the brick's first point (all earlier bricks are full
  // along the dims before the last partial one)
  const uint64_t brick_base = (uint64_t)(bx.o0 * a.g.n[1] * a.g.n[2] + bx.Eb0 * bx.o1 * a.g.n[2] +
                                         bx.Eb0 * bx.Eb1 * bx.o2);
  const uint32_t nbrick = (uint32_t)bx.Eb0 * bx.Eb1 * bx.Eb2;
  const uint32_t nbox = (uint32_t)bx.E0 * bx.b0;
  const uint32_t mgb0 = fmagic((uint32_t)bx.b0), mgE2 = fmagic((uint32_t)bx.E2);
  const int a0 = a.g.act[0], a1 = a.g.act[1], a2 = a.g.act[2];

  // load: faces from the face arrays, interiors from X (compress)
  const T* __restrict__ F0 = reinterpret_cast<const T*>(f.val[0]);
  const T* __restrict__ F1 = reinterpret_cast<const T*>(f.val[1]);
  const T* __restrict__ F2 = reinterpret_cast<const T*>(f.val[2]);
  // eight loads in flight per lane before their LDS stores
  constexpr int kU = 8;
  for (uint32_t i0 = threadIdx.x; i0 < nbox; i0 += kU * blockDim.x) {
    T v[kU];
#pragma unroll
    for (int u = 0; u < kU; u++) {
      const uint32_t i = i0 + u * blockDim.x;
      v[u] = (T)0;
      if (i >= nbox) continue;
      const int32_t c0 = (int32_t)fdiv(i, mgb0);
      const uint32_t rem = i - (uint32_t)c0 * bx.b0;
      const int32_t c1 = (int32_t)fdiv(rem, mgE2);
      const int32_t c2 = (int32_t)(rem - (uint32_t)c1 * bx.E2);
      const int64_t x0 = bx.o0 + c0, x1 = bx.o1 + c1, x2 = bx.o2 + c2;
      if (a0 && (c0 == 0 || c0 == kBrick)) {
        v[u] = F0[(x0 >> f.blog2) * f.plane[0] + x1 * f.fs[0][1] + x2 * f.fs[0][2]];
      } else if (a1 && (c1 == 0 || c1 == kBrick)) {
        v[u] = F1[(x1 >> f.blog2) * f.plane[1] + x0 * f.fs[1][0] + x2 * f.fs[1][2]];
      } else if (a2 && (c2 == 0 || c2 == kBrick)) {
        v[u] = F2[(x2 >> f.blog2) * f.plane[2] + x0 * f.fs[2][0] + x1 * f.fs[2][1]];
      } else if (MODE == 0) {
        v[u] = X[x0 * st0 + x1 * st1 + x2];
      }
    }
#pragma unroll
    for (int u = 0; u < kU; u++) {
      const uint32_t i = i0 + u * blockDim.x;
      if (i < nbox) L[i] = v[u];
    }
  }
  __syncthreads();

  const hpez_interp c = a.cand[bcfg[bi]];
  const int nact = a0 + a1 + a2;
  for (int l = a.L; l >= 1; l--) {
    const int32_t s = 1 << (l - 1);
    const double el = a.el_l[l], inv2e = a.inv2e_l[l], twoe = a.twoe_l[l];
    if (c.md) {
      for (int cnt = 1; cnt <= nact; cnt++) {
        for (unsigned odd = 1; odd < 8; odd++) {
          if ((int)__popc(odd) != cnt) continue;
          if (((odd & 1u) && !a0) || ((odd & 2u) && !a1) || ((odd & 4u) && !a2)) continue;
          const int32_t r0 = (odd & 1u) ? s : 0, r1 = (odd & 2u) ? s : 0, r2 = (odd & 4u) ? s : 0;
          const int32_t m0 = a0 ? 2 * s : 1, m1 = a1 ? 2 * s : 1, m2 = a2 ? 2 * s : 1;
          interior_step<T, MODE>(a, bx, L, r0, r1, r2, m0, m1, m2, c.kind, 0, -1, odd, s, el, inv2e,
                                 twoe, wq, code, brick_base, out);
        }
        __syncthreads();
      }
    } else {
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
      unsigned earlier = 0;  // dims of earlier passes: multiples of s; later: of 2s
      for (int k = 0; k < np; k++) {
        const int pd = (int)(pds >> (2 * k) & 3u);
        int32_t r0 = 0, r1 = 0, r2 = 0;
        int32_t m0 = !a0 ? 1 : ((earlier & 1u) ? s : 2 * s);
        int32_t m1 = !a1 ? 1 : ((earlier & 2u) ? s : 2 * s);
        int32_t m2 = !a2 ? 1 : ((earlier & 4u) ? s : 2 * s);
        if (c.kind != 0 && c.same_level) {
          for (int half = 0; half < 2; half++) {
            const int32_t rh = half ? 3 * s : s;
            if (pd == 0) { r0 = rh; m0 = 4 * s; }
            if (pd == 1) { r1 = rh; m1 = 4 * s; }
            if (pd == 2) { r2 = rh; m2 = 4 * s; }
            interior_step<T, MODE>(a, bx, L, r0, r1, r2, m0, m1, m2, c.kind, half, pd, 0, s, el,
                                   inv2e, twoe, wq, code, brick_base, out);
            __syncthreads();
          }
        } else {
          if (pd == 0) { r0 = s; m0 = 2 * s; }
          if (pd == 1) { r1 = s; m1 = 2 * s; }
          if (pd == 2) { r2 = s; m2 = 2 * s; }
          interior_step<T, MODE>(a, bx, L, r0, r1, r2, m0, m1, m2, c.kind, 0, pd, 0, s, el, inv2e,
                                 twoe, wq, code, brick_base, out);
          __syncthreads();
        }
        earlier |= 1u << pd;
      }
    }
  }

  const uint32_t mgEb12 = fmagic((uint32_t)(bx.Eb1 * bx.Eb2)), mgEb2 = fmagic((uint32_t)bx.Eb2);
  const uint32_t Eb12 = (uint32_t)(bx.Eb1 * bx.Eb2);
  if (MODE == 1) {
    // the whole brick (interiors from the schedule, near faces as loaded)
    for (uint32_t i = threadIdx.x; i < nbrick; i += blockDim.x) {
      const uint32_t c0 = fdiv(i, mgEb12);
      const uint32_t rem = i - c0 * Eb12;
      const uint32_t c1 = fdiv(rem, mgEb2);
      const uint32_t c2 = rem - c1 * (uint32_t)bx.Eb2;
      out[(bx.o0 + c0) * st0 + (bx.o1 + c1) * st1 + (bx.o2 + c2)] =
          L[c0 * bx.b0 + c1 * bx.b1 + c2];
    }
    return;
  }

  // near-face codes of the brick, from the face arrays
  for (uint32_t i = threadIdx.x; i < nbrick; i += blockDim.x) {
    const uint32_t c0 = fdiv(i, mgEb12);
    const uint32_t rem = i - c0 * Eb12;
    const uint32_t c1 = fdiv(rem, mgEb2);
    const uint32_t c2 = rem - c1 * (uint32_t)bx.Eb2;
    const int64_t x0 = bx.o0 + c0, x1 = bx.o1 + c1, x2 = bx.o2 + c2;
    if (a0 && c0 == 0)
      code[brick_base + i] = f.code[0][(x0 >> f.blog2) * f.plane[0] + x1 * f.fs[0][1] + x2 * f.fs[0][2]];
    else if (a1 && c1 == 0)
      code[brick_base + i] = f.code[1][(x1 >> f.blog2) * f.plane[1] + x0 * f.fs[1][0] + x2 * f.fs[1][2]];
    else if (a2 && c2 == 0)
      code[brick_base + i] = f.code[2][(x2 >> f.blog2) * f.plane[2] + x0 * f.fs[2][0] + x1 * f.fs[2][1]];
  }
  __syncthreads();

  // histogram of the brick's codes: a window around R in LDS (reusing the box)
  uint32_t* h = reinterpret_cast<uint32_t*>(lds_raw);
  for (int i = threadIdx.x; i < kBlockHistWin; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const uint32_t lo = a.hist_lo;
  for (uint32_t i = threadIdx.x; i < nbrick; i += blockDim.x) {
    const uint32_t q = code[brick_base + i];
    const uint32_t w = q - lo;
    if (w < (uint32_t)kBlockHistWin) atomicAdd(&h[w], 1u);
    else atomicAdd(&hist[q], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kBlockHistWin; i += blockDim.x)
    if (h[i]) atomicAdd(&hist[lo + i], h[i]);
}

// ---------------------------------------------------------------------------
static unsigned gridn(uint64_t n)
{
  uint64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  return (unsigned)(b ? b : 1);
}

template <typename T>
hipError_t launch_face_init(const FaceGeo& f, const Geom& g, const Lattice& lat, const T* W,
                            const uint16_t* code, int mode, hipStream_t st)
{
  if (!lat.total) return hipSuccess;
  if (mode == 0)
    hipLaunchKernelGGL((face_init_kernel<T, 0>), dim3(gridn(lat.total)), dim3(256), 0, st, f, g,
                       lat, W, code);
  else
    hipLaunchKernelGGL((face_init_kernel<T, 1>), dim3(gridn(lat.total)), dim3(256), 0, st, f, g,
                       lat, W, code);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_face_step(const FaceStep& a, const FaceGeo& f, const T* X, uint16_t* code,
                            const T* out, int mode, hipStream_t st)
{
  if (!a.total) return hipSuccess;
  if (mode == 0)
    hipLaunchKernelGGL((face_step_kernel<T, 0>), dim3(gridn(a.total)), dim3(256), 0, st, a, f, X,
                       code, out);
  else
    hipLaunchKernelGGL((face_step_kernel<T, 1>), dim3(gridn(a.total)), dim3(256), 0, st, a, f, X,
                       code, out);
  return hipGetLastError();
}

template <typename T>
size_t block_lds_bytes(const Geom& g)
{
  size_t pts = 1;
  for (int d = 0; d < 4; d++) {
    const int64_t e = g.act[d] ? kBrick + 1 : kBrick;
    pts *= (size_t)(g.n[d] < e ? g.n[d] : e);
  }
  size_t b = pts * sizeof(T);
  const size_t hb = (size_t)kBlockHistWin * 4;
  return b > hb ? b : hb;
}

template <typename T>
hipError_t launch_blocks(const BlockArgs& a, const FaceGeo& f, const T* X, uint16_t* code,
                         const uint8_t* d_bcfg, const double* d_wq, uint32_t* hist, T* out,
                         int mode, hipStream_t st)
{
  uint64_t nbt = 1;
  for (int d = 0; d < 4; d++) nbt *= (uint64_t)a.nb[d];
  if (!nbt) return hipSuccess;
  const size_t lds = block_lds_bytes<T>(a.g);
  if (mode == 0) {
    (void)hipFuncSetAttribute((const void*)block_kernel<T, 0>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((block_kernel<T, 0>), dim3((unsigned)nbt), dim3(1024), lds, st, a, f, X, code,
                       d_bcfg, d_wq, hist, out);
  } else {
    (void)hipFuncSetAttribute((const void*)block_kernel<T, 1>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((block_kernel<T, 1>), dim3((unsigned)nbt), dim3(1024), lds, st, a, f, X, code,
                       d_bcfg, d_wq, hist, out);
  }
  return hipGetLastError();
}

#define INST(T)                                                                                  \
  template hipError_t launch_face_init<T>(const FaceGeo&, const Geom&, const Lattice&, const T*, \
                                          const uint16_t*, int, hipStream_t);                    \
  template hipError_t launch_face_step<T>(const FaceStep&, const FaceGeo&, const T*, uint16_t*,  \
                                          const T*, int, hipStream_t);                           \
  template size_t block_lds_bytes<T>(const Geom&);                                               \
  template hipError_t launch_blocks<T>(const BlockArgs&, const FaceGeo&, const T*, uint16_t*,     \
                                       const uint8_t*, const double*, uint32_t*, T*, int,        \
                                       hipStream_t);
INST(float)
INST(double)

}  // namespace hpez
