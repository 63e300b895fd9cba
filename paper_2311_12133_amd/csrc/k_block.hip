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
#include "box_dev.h"
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

// one step of the face phase for every family it touches; I is the index
// type (32-bit when the launch has fewer than 2^32 points)
template <typename T, int MODE, typename I>
__global__ void __launch_bounds__(256) face_step_kernel(FaceStep a, FaceGeo f,
                                                        const T* __restrict__ X,
                                                        uint16_t* __restrict__ code,
                                                        const T* __restrict__ out)
{
  const I total = (I)a.off[4];
  const I stride = (I)gridDim.x * blockDim.x;
  for (I k = (I)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += stride) {
    int d = 0;
    if ((uint64_t)k >= a.off[1]) d = 1;
    if ((uint64_t)k >= a.off[2]) d = 2;
    if ((uint64_t)k >= a.off[3]) d = 3;
    // plane index slowest, other dims row-major (last dim fastest)
    int64_t x[4];
    I r = k - (I)a.off[d];
#pragma unroll
    for (int e = 3; e >= 0; e--) {
      if (e == d) continue;
      const I c = (I)a.cnt[e];
      const I q = r / c;
      x[e] = a.first[e] + (int64_t)(r - q * c) * a.step[e];
      r = q;
    }
    x[d] = (int64_t)r * f.B;
    bool skip = false;
#pragma unroll
    for (int e = 0; e < 3; e++)
      if (e < d && a.g.act[e] && (x[e] & (f.B - 1)) == 0) skip = true;  // belongs to family e
    if (skip) continue;
    const T* __restrict__ F = reinterpret_cast<const T*>(f.val[d]);
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
// The grid has at most three dims here (dims 0..2; dim 3 has size 1).

struct Block3 {
  int64_t o0, o1, o2;      // block origin
  int32_t Eb0, Eb1, Eb2;   // brick extents
};

__device__ __forceinline__ void block_geometry(const Geom& g, int64_t bi, const int64_t* nb,
                                               Block3& k, Box& bx)
{
  const int64_t q2 = bi / nb[2];
  const int64_t i2 = bi - q2 * nb[2];
  const int64_t i0 = q2 / nb[1];
  const int64_t i1 = q2 - i0 * nb[1];
  k.o0 = i0 * kBrick;
  k.o1 = i1 * kBrick;
  k.o2 = i2 * kBrick;
  const int64_t r0 = g.n[0] - k.o0, r1 = g.n[1] - k.o1, r2 = g.n[2] - k.o2;
  k.Eb0 = (int32_t)(r0 < kBrick ? r0 : kBrick);
  k.Eb1 = (int32_t)(r1 < kBrick ? r1 : kBrick);
  k.Eb2 = (int32_t)(r2 < kBrick ? r2 : kBrick);
  // closed box along active dims (the far faces belong to the next blocks)
  bx.E0 = g.act[0] ? (int32_t)(r0 < kBrick + 1 ? r0 : kBrick + 1) : k.Eb0;
  bx.E1 = g.act[1] ? (int32_t)(r1 < kBrick + 1 ? r1 : kBrick + 1) : k.Eb1;
  bx.E2 = g.act[2] ? (int32_t)(r2 < kBrick + 1 ? r2 : kBrick + 1) : k.Eb2;
  bx.b1 = bx.E2;
  bx.b0 = bx.E1 * bx.E2;
  bx.a0 = g.act[0];
  bx.a1 = g.act[1];
  bx.a2 = g.act[2];
  // interiors: coordinate 0 is a face along active dims
  bx.lo0 = bx.a0;
  bx.lo1 = bx.a1;
  bx.lo2 = bx.a2;
  bx.hi0 = k.Eb0 - 1;
  bx.hi1 = k.Eb1 - 1;
  bx.hi2 = k.Eb2 - 1;
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
  Block3 bk;
  Box bx;
  block_geometry(a.g, bi, a.nb, bk, bx);
  const int64_t st0 = a.g.st[0], st1 = a.g.st[1];
  // stream position of the brick's first point (all earlier bricks are full
  // along the dims before the last partial one)
  const uint64_t brick_base = (uint64_t)(bk.o0 * a.g.n[1] * a.g.n[2] + bk.Eb0 * bk.o1 * a.g.n[2] +
                                         bk.Eb0 * bk.Eb1 * bk.o2);
  const uint32_t nbrick = (uint32_t)bk.Eb0 * bk.Eb1 * bk.Eb2;
  const uint32_t nbox = (uint32_t)bx.E0 * bx.b0;
  const uint32_t mgb0 = fmagic((uint32_t)bx.b0), mgE2 = fmagic((uint32_t)bx.E2);
  const int a0 = bx.a0, a1 = bx.a1, a2 = bx.a2;

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
      const int64_t x0 = bk.o0 + c0, x1 = bk.o1 + c1, x2 = bk.o2 + c2;
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
  const uint32_t R = a.R;
  const int32_t Eb1 = bk.Eb1, Eb2 = bk.Eb2;
  for (int l = a.L; l >= 1; l--) {
    const int32_t s = 1 << (l - 1);
    const double el = a.el_l[l], inv2e = a.inv2e_l[l], twoe = a.twoe_l[l];
    if (MODE == 0) {
      auto op = [&](int32_t li, int32_t x0, int32_t x1, int32_t x2, T p) {
        const T xv = L[li];
        T xr = xv;
        const uint32_t q = quantize<T>(xv, p, inv2e, twoe, el, R, xr);
        code[brick_base + (uint32_t)((x0 * Eb1 + x1) * Eb2 + x2)] = (uint16_t)q;
        L[li] = q ? xr : xv;
      };
      box_level<T>(c, bx, L, bk.o0, bk.o1, bk.o2, s, wq, op);
    } else {
      auto op = [&](int32_t li, int32_t x0, int32_t x1, int32_t x2, T p) {
        const uint32_t q = code[brick_base + (uint32_t)((x0 * Eb1 + x1) * Eb2 + x2)];
        L[li] = q ? (T)((double)p + (double)((int64_t)q - (int64_t)R) * twoe)
                  : out[(bk.o0 + x0) * st0 + (bk.o1 + x1) * st1 + (bk.o2 + x2)];
      };
      box_level<T>(c, bx, L, bk.o0, bk.o1, bk.o2, s, wq, op);
    }
  }

  const uint32_t mgEb12 = fmagic((uint32_t)(bk.Eb1 * bk.Eb2)), mgEb2 = fmagic((uint32_t)bk.Eb2);
  const uint32_t Eb12 = (uint32_t)(bk.Eb1 * bk.Eb2);
  if (MODE == 1) {
    // the whole brick (interiors from the schedule, near faces as loaded)
    for (uint32_t i = threadIdx.x; i < nbrick; i += blockDim.x) {
      const uint32_t c0 = fdiv(i, mgEb12);
      const uint32_t rem = i - c0 * Eb12;
      const uint32_t c1 = fdiv(rem, mgEb2);
      const uint32_t c2 = rem - c1 * (uint32_t)bk.Eb2;
      out[(bk.o0 + c0) * st0 + (bk.o1 + c1) * st1 + (bk.o2 + c2)] =
          L[c0 * bx.b0 + c1 * bx.b1 + c2];
    }
    return;
  }

  // near-face codes of the brick, from the face arrays
  for (uint32_t i = threadIdx.x; i < nbrick; i += blockDim.x) {
    const uint32_t c0 = fdiv(i, mgEb12);
    const uint32_t rem = i - c0 * Eb12;
    const uint32_t c1 = fdiv(rem, mgEb2);
    const uint32_t c2 = rem - c1 * (uint32_t)bk.Eb2;
    const int64_t x0 = bk.o0 + c0, x1 = bk.o1 + c1, x2 = bk.o2 + c2;
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
  // every lane of the work-group runs the same trip count (wave-level aggregation)
  for (uint32_t i0 = 0; i0 < nbrick; i0 += blockDim.x) {
    const uint32_t i = i0 + threadIdx.x;
    const bool ok = i < nbrick;
    const uint32_t q = ok ? code[brick_base + i] : 0u;
    hist_add_wave(h, hist, lo, (uint32_t)kBlockHistWin, q, ok);
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
  const uint64_t total = a.off[4];
  if (!total) return hipSuccess;
  const dim3 grid(gridn(total)), block(256);
  const bool narrow = total < (1ull << 32);
  if (mode == 0 && narrow)
    hipLaunchKernelGGL((face_step_kernel<T, 0, uint32_t>), grid, block, 0, st, a, f, X, code, out);
  else if (mode == 0)
    hipLaunchKernelGGL((face_step_kernel<T, 0, uint64_t>), grid, block, 0, st, a, f, X, code, out);
  else if (narrow)
    hipLaunchKernelGGL((face_step_kernel<T, 1, uint32_t>), grid, block, 0, st, a, f, X, code, out);
  else
    hipLaunchKernelGGL((face_step_kernel<T, 1, uint64_t>), grid, block, 0, st, a, f, X, code, out);
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
