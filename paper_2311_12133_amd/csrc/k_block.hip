// k_block.hip -- block-wise interpolation on MI355X (Sec. 6.6 configurations,
// Sec. 5 predictor), for block side B = 32 (the paper's default, equal to the
// stream's brick side).
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
// interiors: one work-group per block, the whole schedule below B in LDS

struct BoxGeo {
  int64_t o[4];    // block origin
  int32_t E[4];    // box extents (closed box along active dims)
  int32_t bs[4];   // LDS strides
  int32_t hi[4];   // last interior coordinate (box-local)
  int32_t Eb[4];   // brick extents (half-open)
};

__device__ __forceinline__ void box_setup(const Geom& g, int64_t bi, const int64_t* nb, BoxGeo& bx)
{
  int64_t r = bi;
  int64_t b[4];
  for (int d = 3; d >= 0; d--) {
    b[d] = r % nb[d];
    r /= nb[d];
  }
  for (int d = 0; d < 4; d++) {
    bx.o[d] = b[d] * kBrick;
    const int64_t rem = g.n[d] - bx.o[d];
    bx.Eb[d] = (int32_t)(rem < kBrick ? rem : kBrick);
    if (g.act[d]) {
      bx.E[d] = (int32_t)(rem < kBrick + 1 ? rem : kBrick + 1);
      bx.hi[d] = (int32_t)(rem - 1 < kBrick - 1 ? rem - 1 : kBrick - 1);
    } else {
      bx.E[d] = bx.Eb[d];
      bx.hi[d] = bx.Eb[d] - 1;
    }
  }
  bx.bs[3] = 1;
  for (int d = 2; d >= 0; d--) bx.bs[d] = bx.bs[d + 1] * bx.E[d + 1];
}

// smallest c in [lo, ...] with (o + c) == r (mod m)
__device__ __forceinline__ int32_t first_in(int64_t o, int32_t lo, int64_t r, int64_t m)
{
  const int64_t x0 = o + lo;
  int64_t v = x0 - ((x0 - r) % m + m) % m;
  if (v < x0) v += m;
  return (int32_t)(v - o);
}

template <typename T, int MODE>
__device__ void interior_step(const BlockArgs& a, const BoxGeo& bx, T* L, const int64_t* r,
                              const int64_t* m, const hpez_interp& c, int sl, int pd, unsigned odd,
                              int64_t s, double el, double inv2e, double twoe,
                              const double* __restrict__ wq, uint16_t* __restrict__ code,
                              uint64_t brick_base, const T* __restrict__ out)
{
  int32_t f[4], cnt[4], mm[4];
  uint32_t total = 1;
  for (int d = 0; d < 4; d++) {
    const int32_t lo = a.g.act[d] ? 1 : 0;
    mm[d] = (int32_t)m[d];
    f[d] = first_in(bx.o[d], lo, r[d], m[d]);
    cnt[d] = f[d] <= bx.hi[d] ? (bx.hi[d] - f[d]) / mm[d] + 1 : 0;
    total *= (uint32_t)cnt[d];
  }
  for (uint32_t k = threadIdx.x; k < total; k += blockDim.x) {
    int32_t cc[4];
    uint32_t rr = k;
    for (int d = 3; d >= 0; d--) {
      const uint32_t q = rr / (uint32_t)cnt[d];
      cc[d] = f[d] + (int32_t)(rr - q * (uint32_t)cnt[d]) * mm[d];
      rr = q;
    }
    const int32_t li = cc[0] * bx.bs[0] + cc[1] * bx.bs[1] + cc[2] * bx.bs[2] + cc[3];
    T p;
    if (!c.md) {
      p = spline<T, T>(L, li, s * bx.bs[pd], cc[pd], s, 0, bx.E[pd] - 1, c.kind, sl);
    } else {
      bool first = true;
      T acc = (T)0;
      for (int d = 0; d < 4; d++) {
        if (!(odd >> d & 1u)) continue;
        const T pv = spline<T, T>(L, li, s * bx.bs[d], cc[d], s, 0, bx.E[d] - 1, c.kind, 0);
        const T term = (T)wq[(c.kind * 16 + odd) * 4 + d] * pv;
        acc = first ? term : acc + term;
        first = false;
      }
      p = acc;
    }
    const uint64_t cpos =
        brick_base + (uint64_t)(((cc[0] * bx.Eb[1] + cc[1]) * bx.Eb[2] + cc[2]) * bx.Eb[3] + cc[3]);
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
        const int64_t idx = (bx.o[0] + cc[0]) * a.g.st[0] + (bx.o[1] + cc[1]) * a.g.st[1] +
                            (bx.o[2] + cc[2]) * a.g.st[2] + (bx.o[3] + cc[3]);
        L[li] = out[idx];
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
  BoxGeo bx;
  box_setup(a.g, bi, a.nb, bx);
  const int32_t nbox = bx.bs[0] * bx.E[0];
  // brick base: stream position of the brick's first point
  int64_t b0[4];
  for (int d = 0; d < 4; d++) b0[d] = bx.o[d];
  const uint64_t brick_base = (uint64_t)brick_pos(a.g.n, b0);
  const uint32_t nbrick = (uint32_t)bx.Eb[0] * bx.Eb[1] * bx.Eb[2] * bx.Eb[3];

  // load: faces from the face arrays, interiors from X (compress)
  for (int32_t i = threadIdx.x; i < nbox; i += blockDim.x) {
    int32_t cc[4], rr = i;
    for (int d = 3; d >= 0; d--) {
      cc[d] = rr % bx.E[d];
      rr /= bx.E[d];
    }
    int fam = -1;
    for (int d = 0; d < 4; d++)
      if (a.g.act[d] && (cc[d] == 0 || cc[d] == kBrick)) {
        fam = d;
        break;
      }
    int64_t x[4];
    for (int d = 0; d < 4; d++) x[d] = bx.o[d] + cc[d];
    if (fam >= 0) {
      L[i] = reinterpret_cast<const T*>(f.val[fam])[face_index(f, fam, x)];
    } else if (MODE == 0) {
      L[i] = X[x[0] * a.g.st[0] + x[1] * a.g.st[1] + x[2] * a.g.st[2] + x[3]];
    }
  }
  __syncthreads();

  const hpez_interp c = a.cand[bcfg[bi]];
  int nact = 0;
  for (int d = 0; d < 4; d++) nact += a.g.act[d];
  for (int l = a.L; l >= 1; l--) {
    const int64_t s = (int64_t)1 << (l - 1);
    const double el = a.el_l[l], inv2e = a.inv2e_l[l], twoe = a.twoe_l[l];
    int64_t r[4], m[4];
    if (c.md) {
      for (int cnt = 1; cnt <= nact; cnt++) {
        for (unsigned odd = 1; odd < 16; odd++) {
          bool ok = __popc(odd) == cnt;
          for (int d = 0; d < 4; d++)
            if ((odd >> d & 1u) && !a.g.act[d]) ok = false;
          if (!ok) continue;
          for (int d = 0; d < 4; d++) {
            if (!a.g.act[d]) { r[d] = 0; m[d] = 1; }
            else if (odd >> d & 1u) { r[d] = s; m[d] = 2 * s; }
            else { r[d] = 0; m[d] = 2 * s; }
          }
          interior_step<T, MODE>(a, bx, L, r, m, c, 0, -1, odd, s, el, inv2e, twoe, wq, code,
                                 brick_base, out);
        }
        __syncthreads();
      }
    } else {
      int pos[4] = {-1, -1, -1, -1}, np = 0;
      for (int i = 0; i < 4; i++) {
        const int d = c.order[i];
        if (d < 4 && a.g.act[d] && pos[d] < 0) pos[d] = np++;
      }
      for (int k = 0; k < np; k++) {
        int pd = 0;
        for (int d = 0; d < 4; d++)
          if (pos[d] == k) pd = d;
        for (int d = 0; d < 4; d++) {
          if (!a.g.act[d]) { r[d] = 0; m[d] = 1; }
          else if (d == pd) { r[d] = s; m[d] = 2 * s; }
          else if (pos[d] < k) { r[d] = 0; m[d] = s; }
          else { r[d] = 0; m[d] = 2 * s; }
        }
        if (c.kind != 0 && c.same_level) {
          m[pd] = 4 * s;
          r[pd] = s;
          interior_step<T, MODE>(a, bx, L, r, m, c, 0, pd, 0, s, el, inv2e, twoe, wq, code,
                                 brick_base, out);
          __syncthreads();
          r[pd] = 3 * s;
          interior_step<T, MODE>(a, bx, L, r, m, c, 1, pd, 0, s, el, inv2e, twoe, wq, code,
                                 brick_base, out);
        } else {
          interior_step<T, MODE>(a, bx, L, r, m, c, 0, pd, 0, s, el, inv2e, twoe, wq, code,
                                 brick_base, out);
        }
        __syncthreads();
      }
    }
  }

  if (MODE == 1) {
    // the whole brick (interiors from the schedule, near faces as loaded)
    for (uint32_t i = threadIdx.x; i < nbrick; i += blockDim.x) {
      int32_t cc[4];
      uint32_t rr = i;
      for (int d = 3; d >= 0; d--) {
        cc[d] = (int32_t)(rr % (uint32_t)bx.Eb[d]);
        rr /= (uint32_t)bx.Eb[d];
      }
      const int32_t li = cc[0] * bx.bs[0] + cc[1] * bx.bs[1] + cc[2] * bx.bs[2] + cc[3];
      out[(bx.o[0] + cc[0]) * a.g.st[0] + (bx.o[1] + cc[1]) * a.g.st[1] +
          (bx.o[2] + cc[2]) * a.g.st[2] + (bx.o[3] + cc[3])] = L[li];
    }
    return;
  }

  // near-face codes of the brick, from the face arrays
  for (uint32_t i = threadIdx.x; i < nbrick; i += blockDim.x) {
    int32_t cc[4];
    uint32_t rr = i;
    for (int d = 3; d >= 0; d--) {
      cc[d] = (int32_t)(rr % (uint32_t)bx.Eb[d]);
      rr /= (uint32_t)bx.Eb[d];
    }
    int fam = -1;
    for (int d = 0; d < 4; d++)
      if (a.g.act[d] && cc[d] == 0) {
        fam = d;
        break;
      }
    if (fam < 0) continue;
    int64_t x[4];
    for (int d = 0; d < 4; d++) x[d] = bx.o[d] + cc[d];
    code[brick_base + i] = f.code[fam][face_index(f, fam, x)];
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
