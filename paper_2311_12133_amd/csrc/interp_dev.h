// interp_dev.h -- device-side spline stencils and quantizer shared by the
// predictor kernels and the tuner's trial kernels (gfx950).
//
// Floating point: the stencils are evaluated in T in the order written, the
// quantizer in double; the library is built with -ffp-contract=off so no
// operation is fused.
#pragma once

#include "hpez_internal.h"

namespace hpez {

// Pointers into device global memory.  Accesses through them compile to
// global_* instructions.  Through a generic pointer the compiler must emit
// flat_* instructions (e.g. for pointers read from a table in memory), and a
// flat access also counts against the LDS wait counter: every later LDS wait
// would then wait for outstanding global loads and stores as well.
#define HPEZ_GLOBAL __attribute__((address_space(1)))
#ifdef __HIPCC__
template <typename T>
__device__ __forceinline__ HPEZ_GLOBAL T* gmem(T* p)
{
  return (HPEZ_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ const HPEZ_GLOBAL T* gmem(const T* p)
{
  return (const HPEZ_GLOBAL T*)p;
}
#endif

template <typename T>
struct SplineK;
template <>
struct SplineK<float> {
  static __device__ __forceinline__ float k6() { return 0x1.555556p-3f; }
  static __device__ __forceinline__ float k40() { return 0x1.99999ap-6f; }
  static __device__ __forceinline__ float k62() { return 0x1.084210p-6f; }
};
template <>
struct SplineK<double> {
  static __device__ __forceinline__ double k6() { return 0x1.5555555555555p-3; }
  static __device__ __forceinline__ double k40() { return 0x1.999999999999ap-6; }
  static __device__ __forceinline__ double k62() { return 0x1.0842108421084p-6; }
};

// One-dimensional spline prediction along a dimension with index step sd = s *
// stride, for a point at coordinate x whose usable neighbours lie in [lo, hi].
// Interior stencils: Eq. (2) linear, Eq. (6) not-a-knot, Eq. (8) natural,
// Eq. (13)/(14) same-level.  At the grid (or block) end the Lagrange polynomial
// through the neighbours that exist is used.
template <typename T, typename P>
__device__ __forceinline__ T spline(const P* __restrict__ W, int64_t idx, int64_t sd, int64_t x,
                                    int64_t s, int64_t lo, int64_t hi, int kind, int sl)
{
  const bool ha = x - 3 * s >= lo;
  const bool hc = x + s <= hi;
  const bool hd = x + 3 * s <= hi;
  const T b = W[idx - sd];
  if (kind == 0) {
    if (hc) return (b + (T)W[idx + sd]) * (T)0.5;
    if (ha) return (b * (T)3 - (T)W[idx - 3 * sd]) * (T)0.5;
    return b;
  }
  if (sl) {
    const bool ha2 = x - 2 * s >= lo;
    const bool hd2 = x + 2 * s <= hi;
    if (kind == 1 && ha2 && hc && hd2)
      return ((b + (T)W[idx + sd]) * (T)4 - ((T)W[idx - 2 * sd] + (T)W[idx + 2 * sd])) *
             SplineK<T>::k6();
    if (kind == 2 && ha && ha2 && hc && hd2 && hd)
      return ((b + (T)W[idx + sd]) * (T)46 - ((T)W[idx - 2 * sd] + (T)W[idx + 2 * sd]) * (T)18 +
              ((T)W[idx - 3 * sd] + (T)W[idx + 3 * sd]) * (T)3) *
             SplineK<T>::k62();
  }
  if (ha && hc && hd) {
    const T a = W[idx - 3 * sd], c = W[idx + sd], d = W[idx + 3 * sd];
    if (kind == 1) return ((b + c) * (T)9 - (a + d)) * (T)0.0625;
    return ((b + c) * (T)23 - (a + d) * (T)3) * SplineK<T>::k40();
  }
  if (hc && hd) return (b * (T)3 + (T)W[idx + sd] * (T)6 - (T)W[idx + 3 * sd]) * (T)0.125;
  if (ha && hc) return (b * (T)6 + (T)W[idx + sd] * (T)3 - (T)W[idx - 3 * sd]) * (T)0.125;
  if (hc) return (b + (T)W[idx + sd]) * (T)0.5;
  if (ha) return (b * (T)3 - (T)W[idx - 3 * sd]) * (T)0.5;
  return b;
}

// Checkerboard colour of a point of a multi-dimensional sub-step with odd set
// `odd` at stride s (a power of two): the parity of sum (x_d - s) / 2s over the
// odd dims.  Same-level cubic inside MD (Sec. 5.4.2) predicts colour 0 with the
// regular stencils, then colour 1 with the same-level ones (its neighbours at
// +-2s along an odd dim have colour 0).
__device__ __forceinline__ int md_colour(const int64_t* x, unsigned odd, int64_t s)
{
  int64_t t = 0;
  for (int d = 0; d < 4; d++)
    if (odd >> d & 1u) t += x[d] / (2 * s);
  return (int)(t & 1);
}

// The value rebuilt from prediction p and quantization index qd: p + qd 2e_l
// in double.  A negative twoe marks an integer field (the method then runs in
// double on the integer values): the value is rounded to the nearest integer
// (ties to even), so the working grid holds exactly what the integer output
// will.
template <typename T>
__device__ __forceinline__ T recon(T p, double qd, double twoe)
{
  if constexpr (sizeof(T) == 4) {
    // float kernels never see an integer field (those run in double): twoe > 0
    return (T)((double)p + qd * twoe);
  } else {
    const double v = (double)p + qd * fabs(twoe);
    return (T)(twoe < 0 ? rint(v) : v);
  }
}

// Linear-scale quantization (Sec. 4, step 3): bins of width 2 e_l, rounding
// half away from zero, radius R, double arithmetic; the value the decompressor
// will rebuild (recon) must meet the bound or the point is stored verbatim
// (code 0).
template <typename T>
__device__ __forceinline__ uint32_t quantize(T x, T p, double inv2e, double twoe, double el,
                                             uint32_t R, T& xr)
{
  // evaluated without branches: both checks are computed and select the result
  const double t = ((double)x - (double)p) * inv2e;
  const double qf = floor(fabs(t) + 0.5);
  const bool inr = qf < (double)R;
  const double q = t < 0 ? -qf : qf;
  const T r = recon<T>(p, q, twoe);
  const bool ok = inr && fabs((double)r - (double)x) <= el;
  xr = ok ? r : xr;
  // |q| < R <= 2^15: the 32-bit conversion is exact; code 0 when not ok
  const double qs = ok ? q : -(double)R;
  return (uint32_t)((int32_t)qs + (int32_t)R);
}

// Stream (code) order: bricks of kBrick points per dimension, clipped at the
// grid end, in row-major order; points of a brick in row-major order.
constexpr int64_t kBrick = 1 << kBrickLog2;

__host__ __device__ __forceinline__ int64_t brick_ext(int64_t n, int64_t b)
{
  const int64_t r = n - b * kBrick;
  return r < kBrick ? r : kBrick;
}

// stream position of the point with coordinates x in a grid of dims n
__host__ __device__ __forceinline__ int64_t brick_pos(const int64_t* n, const int64_t* x)
{
  int64_t b[4], c[4], E[4];
  for (int d = 0; d < 4; d++) {
    b[d] = x[d] >> kBrickLog2;
    c[d] = x[d] & (kBrick - 1);
    E[d] = brick_ext(n[d], b[d]);
  }
  return kBrick * b[0] * (n[1] * n[2] * n[3]) + E[0] * kBrick * b[1] * (n[2] * n[3]) +
         E[0] * E[1] * kBrick * b[2] * n[3] + E[0] * E[1] * E[2] * kBrick * b[3] +
         ((c[0] * E[1] + c[1]) * E[2] + c[2]) * E[3] + c[3];
}

// inverse of brick_pos: coordinates of the point at stream position pos
__host__ __device__ __forceinline__ void brick_coords(const int64_t* n, int64_t pos, int64_t* x)
{
  int64_t b[4], E[4], r = pos;
  int64_t above = 1;  // product of extents of the brick slabs already fixed
  for (int d = 0; d < 4; d++) {
    int64_t tail = 1;
    for (int e = d + 1; e < 4; e++) tail *= n[e];
    const int64_t slab = above * kBrick * tail;
    b[d] = r / slab;
    r -= b[d] * slab;
    E[d] = brick_ext(n[d], b[d]);
    above *= E[d];
  }
  // r is the row-major index inside the brick of extents E
  for (int d = 3; d >= 0; d--) {
    x[d] = b[d] * kBrick + r % E[d];
    r /= E[d];
  }
}

// Exact n / d for n, d < 2^16 (so n * d < 2^32) by multiply-high with
// m = ceil(2^32 / d); d = 1 (m = 2^32 does not fit) is stored as 0.  Box
// counts and extents never exceed 33 per dim, so every divisor is at most
// kMagicMax and comes from a table in constant memory.
constexpr uint32_t kMagicMax = 33 * 33 * 9;
struct MagicTable {
  uint32_t m[kMagicMax + 1];
  constexpr MagicTable() : m()
  {
    for (uint32_t d = 2; d <= kMagicMax; d++) m[d] = (uint32_t)(0xFFFFFFFFull / d + 1);
  }
};
__constant__ constexpr MagicTable kDivMagic{};
struct Divisor {
  uint32_t m;     // multiplier (0 for d = 1)
  uint32_t pass;  // all ones for d = 1: the quotient is n itself
};
__device__ __forceinline__ Divisor fmagic(uint32_t d)
{
  const uint32_t m = kDivMagic.m[d];
  return {m, m ? 0u : 0xFFFFFFFFu};
}
// branch-free: one multiply-high, one and, one add
__device__ __forceinline__ uint32_t fdiv(uint32_t n, Divisor d) { return __umulhi(n, d.m) + (n & d.pass); }

// Exact n / d for every 32-bit n and d >= 1 (Granlund and Montgomery's
// round-up multiplier with a shift): q = (t + ((n - t) >> 1)) >> (l - 1) with
// t = mulhi(m, n), l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1; d <= 1
// passes n through (shift -1).  The multiplier needs one 64-bit division, so it
// is made once per work-group or on the host.
struct XDivisor {
  uint32_t m;
  int32_t sh;
};
__host__ __device__ __forceinline__ XDivisor xmagic(uint32_t d)
{
  if (d <= 1) return {0u, -1};
  int l = 0;
  while ((1ull << l) < d) l++;
  return {(uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1), l - 1};
}
__host__ __device__ __forceinline__ uint32_t xdiv(uint32_t n, XDivisor d)
{
  if (d.sh < 0) return n;
  const uint32_t t = (uint32_t)(((uint64_t)d.m * n) >> 32);  // multiply-high
  return (t + ((n - t) >> 1)) >> d.sh;
}

// Histogram update for every lane with `valid`: lanes holding equal codes are
// counted together (one atomic per distinct code in the wavefront), into the
// LDS window [lo, lo + win) or the global table outside it.
__device__ __forceinline__ void hist_add_wave(uint32_t* lh, uint32_t* gh, uint32_t lo, uint32_t win,
                                              uint32_t q, bool valid)
{
  uint64_t pending = __ballot(valid);
  while (pending) {
    const int leader = __builtin_ctzll(pending);
    const uint32_t v = __builtin_amdgcn_readlane(q, leader);
    const uint64_t same = __ballot(valid && q == v) & pending;
    if ((int)(threadIdx.x & 63) == leader) {
      const uint32_t c = (uint32_t)__popcll(same);
      const uint32_t w = v - lo;
      if (w < win) atomicAdd(&lh[w], c);
      else atomicAdd(&gh[v], c);
    }
    pending &= ~same;
  }
}

// v[d] for a run-time d in [0, 4) without indexing a private array (which
// would place the array in scratch memory)
__device__ __forceinline__ int64_t pick4(const int64_t* v, int d)
{
  return d == 0 ? v[0] : d == 1 ? v[1] : d == 2 ? v[2] : v[3];
}

__device__ __forceinline__ void lattice_point(const Lattice& L, uint64_t k, int64_t* x)
{
  uint64_t r = k;
  for (int d = 3; d >= 0; d--) {
    const uint64_t c = L.cnt[d];
    const uint64_t q = r / c;
    x[d] = L.first[d] + (int64_t)(r - q * c) * L.step[d];
    r = q;
  }
}

}  // namespace hpez
