// k_block.hip -- block-wise interpolation on MI355X (Sec. 6.6 configurations,
// Sec. 5 predictor), for block side B = 32 (the paper's default, equal to the
// stream's brick side) and grids of up to three dimensions.
//
// With block-wise configurations, levels with stride s < B are computed in two
// phases (the reading the whole library uses for how blocks meet):
//   * faces: points with some active coordinate a multiple of B, with the
//     level's global configuration.  A face point is never interpolated along
//     the dimension that makes it a face, so every stencil stays inside its
//     face plane.  Face values live in compact per-family arrays (family d =
//     the planes x_d = 0, B, 2B, ...; layout [plane][other dims], so every
//     plane is contiguous); face codes go straight to their stream positions
//     and are counted there;
//   * interiors: one work-group per block runs every level s < B for the
//     block's own configuration, stencils clipped to the block's closed box.
//     The box (B+1)^D lives in LDS and is updated in place: a cell holds the
//     original value until its point is predicted, then the reconstruction.
//     Work-groups are persistent (one per CU, blocks taken from a counter) and
//     load the next block's box into registers while they compute the current
//     one.

#include "block_dev.h"
#include "box_dev.h"
#include "fblock_dev.h"
#include "interp_dev.h"

namespace hpez {

__device__ __forceinline__ int64_t face_index(const FaceGeo& f, int e, const int64_t* x)
{
  int64_t i = (x[e] >> f.blog2) * f.plane[e];
  for (int k = 0; k < 4; k++)
    if (k != e) i += x[k] * f.fs[e][k];
  return i;
}

// index of the last entry whose begin is <= x (begin ascending, begin[0] = 0)
__device__ __forceinline__ int find_entry(const uint64_t* __restrict__ begin, int n, uint64_t x)
{
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// write a face point's value into every family it belongs to
template <typename T>
__device__ __forceinline__ void face_store(const FaceGeo& f, const Geom& g, const int64_t* x, T v)
{
  for (int e = 0; e < 4; e++) {
    if (!g.act[e] || (x[e] & (f.B - 1))) continue;
    gmem(reinterpret_cast<T*>(f.val[e]))[face_index(f, e, x)] = v;
  }
}

// the lowest family a face point belongs to (-1: not on a face)
__device__ __forceinline__ int low_family(const FaceGeo& f, const Geom& g, const int64_t* x)
{
  for (int e = 0; e < 4; e++)
    if (g.act[e] && (x[e] & (f.B - 1)) == 0) return e;
  return -1;
}

// ---------------------------------------------------------------------------
// points on the coarse grid of stride B (anchors and levels s >= B): copy the
// working grid into the face arrays (and, compressing, their codes into the
// code array of their lowest family)
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
    if (MODE == 0) {
      const int e = low_family(f, g, x);
      if (e >= 0) f.code[e][face_index(f, e, x)] = code[brick_pos(g.n, x)];
    }
    face_store<T>(f, g, x, W[idx]);
  }
}

template <typename T>
__device__ __forceinline__ bool face_nonfinite(T v)
{
  return !(v - v == (T)0);
}

// Value range plus face prefill: waves take rows along dim 2; the points with
// x2 on the face lattice (one per 32 values of a row, so a strided read for
// the face steps) go to family 2's face array.  The planes normal to dims 0
// and 1 are contiguous in the field and stay there.  The range is reduced
// exactly as minmax_kernel does.
template <typename T>
__global__ void __launch_bounds__(256) minmax_faces_kernel(const T* __restrict__ X, Geom g, FaceGeo f,
                                                           double* __restrict__ part,
                                                           int* __restrict__ bad)
{
  __shared__ double smn[256], smx[256];
  T mn = X[0], mx = X[0];
  bool nf = false;
  const int lane = threadIdx.x & 63;
  const uint64_t n1 = (uint64_t)g.n[1];
  const int64_t n2 = g.n[2];
  const uint64_t nrows = (uint64_t)g.n[0] * n1;
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t Bm = f.B - 1;
  const bool vec = (n2 & 3) == 0 && ((uintptr_t)X & 15) == 0;
  // four consecutive rows share x0 and their x1 are 4k .. 4k + 3: family 2's
  // values of the four rows are adjacent in its array (one 4-value store)
  const bool quad = (n1 & 3) == 0 && g.act[2];
  if (vec && n2 <= 128 * (int64_t)(16 / sizeof(T))) {
    // rows of at most two vectors per lane: each wave takes 4 consecutive rows and
    // loads all of its vectors of them before using any (8 loads in flight)
    constexpr int V = 16 / sizeof(T);
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    for (uint64_t r0 = wave * 4; r0 < nrows; r0 += nwaves * 4) {
      T t[4][2][V];
#pragma unroll
      for (int u = 0; u < 4; u++)
#pragma unroll
        for (int h = 0; h < 2; h++) {
          const int64_t i = ((int64_t)lane + 64 * h) * V;
          if (r0 + u < nrows && i < n2)
            *reinterpret_cast<u4*>(t[u][h]) =
                *reinterpret_cast<const HPEZ_GLOBAL u4*>(gmem(X) + (r0 + u) * (uint64_t)n2 + i);
        }
      // row coordinates: with n1 a multiple of 4 the four rows share x0 and
      // x1 steps by one (one 32-bit division per four rows; rows < 2^32)
      const uint32_t r0q = (uint32_t)r0 / (uint32_t)n1;
      const uint32_t r0r = (uint32_t)r0 - r0q * (uint32_t)n1;
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const uint64_t r = r0 + u;
        if (r >= nrows) break;
        int64_t x[4] = {0, 0, 0, 0};
        if (quad) {
          x[0] = r0q;
          x[1] = r0r + u;
        } else {
          x[0] = (uint32_t)r / (uint32_t)n1;
          x[1] = (uint32_t)r - (uint32_t)x[0] * (uint32_t)n1;
        }
        HPEZ_GLOBAL T* d2 =
            g.act[2] ? gmem(reinterpret_cast<T*>(f.val[2])) + face_index(f, 2, x) : nullptr;
#pragma unroll
        for (int h = 0; h < 2; h++) {
          const int64_t i = ((int64_t)lane + 64 * h) * V;
          if (i >= n2) continue;
#pragma unroll
          for (int j = 0; j < V; j++) {
            nf |= face_nonfinite(t[u][h][j]);
            mn = t[u][h][j] < mn ? t[u][h][j] : mn;
            mx = t[u][h][j] > mx ? t[u][h][j] : mx;
          }
          if (!quad && d2 && (i & Bm) == 0) d2[(i >> f.blog2) * f.plane[2]] = t[u][h][0];
        }
      }
      if (quad && r0 + 3 < nrows) {
        int64_t x[4] = {(int64_t)r0q, (int64_t)r0r, 0, 0};
        HPEZ_GLOBAL T* d2 = gmem(reinterpret_cast<T*>(f.val[2])) + face_index(f, 2, x);
#pragma unroll
        for (int h = 0; h < 2; h++) {
          const int64_t i = ((int64_t)lane + 64 * h) * V;
          if (i >= n2 || (i & Bm)) continue;
          T q[4] = {t[0][h][0], t[1][h][0], t[2][h][0], t[3][h][0]};
          HPEZ_GLOBAL T* dst = d2 + (i >> f.blog2) * f.plane[2];
          if (sizeof(T) == 4) {
            *reinterpret_cast<HPEZ_GLOBAL u4*>(dst) = *reinterpret_cast<const u4*>(q);
          } else {
            *reinterpret_cast<HPEZ_GLOBAL u4*>(dst) = *reinterpret_cast<const u4*>(q);
            *reinterpret_cast<HPEZ_GLOBAL u4*>(dst + 2) = *reinterpret_cast<const u4*>(q + 2);
          }
        }
      } else if (quad) {
        // the last rows of the field (fewer than four)
        for (int u = 0; u < 4 && r0 + u < nrows; u++) {
          int64_t x[4] = {(int64_t)r0q, (int64_t)r0r + u, 0, 0};
          HPEZ_GLOBAL T* d2 = gmem(reinterpret_cast<T*>(f.val[2])) + face_index(f, 2, x);
#pragma unroll
          for (int h = 0; h < 2; h++) {
            const int64_t i = ((int64_t)lane + 64 * h) * V;
            if (i < n2 && (i & Bm) == 0) d2[(i >> f.blog2) * f.plane[2]] = t[u][h][0];
          }
        }
      }
    }
  } else
  for (uint64_t r = wave; r < nrows; r += nwaves) {
    int64_t x[4] = {(int64_t)(r / n1), (int64_t)(r % n1), 0, 0};
    HPEZ_GLOBAL T* d2 = g.act[2] ? gmem(reinterpret_cast<T*>(f.val[2])) + face_index(f, 2, x) : nullptr;
    const HPEZ_GLOBAL T* row = gmem(X) + r * (uint64_t)n2;
    if (vec) {
      constexpr int V = 16 / sizeof(T);
      for (int64_t i = (int64_t)lane * V; i < n2; i += 64 * V) {
        typedef unsigned int u4 __attribute__((ext_vector_type(4)));
        T t[V];
        *reinterpret_cast<u4*>(t) = *reinterpret_cast<const HPEZ_GLOBAL u4*>(row + i);
#pragma unroll
        for (int j = 0; j < V; j++) {
          nf |= face_nonfinite(t[j]);
          mn = t[j] < mn ? t[j] : mn;
          mx = t[j] > mx ? t[j] : mx;
        }
        if (d2 && (i & Bm) == 0) d2[(i >> f.blog2) * f.plane[2]] = t[0];
      }
    } else {
      for (int64_t i = lane; i < n2; i += 64) {
        const T v = row[i];
        nf |= face_nonfinite(v);
        mn = v < mn ? v : mn;
        mx = v > mx ? v : mx;
        if (d2 && (i & Bm) == 0) d2[(i >> f.blog2) * f.plane[2]] = v;
      }
    }
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

template <typename T>
hipError_t launch_minmax_faces(const T* X, const Geom& g, const FaceGeo& f, double* part, int* bad,
                               int nblocks, hipStream_t st)
{
  hipLaunchKernelGGL((minmax_faces_kernel<T>), dim3(nblocks), dim3(256), 0, st, X, g, f, part, bad);
  return hipGetLastError();
}

// one step of the face phase for every family it touches, for every entry of
// the table (one entry per field); an entry owns a range of work-groups.  I is
// the index type (32-bit when every entry has fewer than 2^32 points).
template <typename T, int MODE, typename I>
__global__ void __launch_bounds__(256) face_step_kernel(const FaceEntry<T>* __restrict__ tab,
                                                        const uint64_t* __restrict__ wg_begin,
                                                        int n)
{
  const int ei = find_entry(wg_begin, n, blockIdx.x);
  const FaceEntry<T>& E = tab[ei];
  const FaceStep& a = E.a;
  const FaceGeo& f = E.f;
  const HPEZ_GLOBAL T* __restrict__ X = gmem(E.X);
  const HPEZ_GLOBAL uint16_t* __restrict__ code = gmem(E.code);
  const HPEZ_GLOBAL T* __restrict__ out = gmem(E.out);
  const I total = (I)a.off[4];
  const I stride = (I)E.wg_count * blockDim.x;
  for (I k = (I)(blockIdx.x - E.wg_begin) * blockDim.x + threadIdx.x; k < total; k += stride) {
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
      I q;
      if constexpr (sizeof(I) == 4) {
        // r / c with the step's magic multiplier (uniform branch on the shift)
        if (a.msh[e] < 0) {
          q = r;
        } else {
          const uint32_t t = __umulhi(a.mg[e], (uint32_t)r);
          q = (t + (((uint32_t)r - t) >> 1)) >> a.msh[e];
        }
      } else {
        q = r / c;
      }
      x[e] = a.first[e] + (int64_t)(r - q * c) * a.step[e];
      r = q;
    }
    x[d] = (int64_t)r * f.B;
    bool skip = false;
#pragma unroll
    for (int e = 0; e < 3; e++)
      if (e < d && a.g.act[e] && (x[e] & (f.B - 1)) == 0) skip = true;  // belongs to family e
    if (skip) continue;
    if (a.md && a.mdhalf && md_colour(x, a.odd, a.s) != a.mdhalf - 1) continue;
    const HPEZ_GLOBAL T* __restrict__ F = gmem(reinterpret_cast<const T*>(f.val[d]));
    const int64_t fi = face_index(f, d, x);
    T p;
    if (!a.md) {
      const int e = a.pdim;
      p = spline<T, HPEZ_GLOBAL T>(F, fi, a.s * f.fs[d][e], x[e], a.s, 0, a.g.n[e] - 1, a.kind,
                                   a.sl);
    } else {
      bool first = true;
      T acc = (T)0;
      for (int e = 0; e < 4; e++) {
        if (!(a.odd >> e & 1u)) continue;
        const T pe = spline<T, HPEZ_GLOBAL T>(F, fi, a.s * f.fs[d][e], x[e], a.s, 0, a.g.n[e] - 1,
                                              a.kind, a.sl);
        const T term = (T)a.wq[e] * pe;
        acc = first ? term : acc + term;
        first = false;
      }
      p = acc;
    }
    const int64_t idx = x[0] * a.g.st[0] + x[1] * a.g.st[1] + x[2] * a.g.st[2] + x[3];
    if (MODE == 0) {
      const T xv = (d == 2 && E.xface) ? F[fi] : X[idx];
      T xr = xv;
      const uint32_t q = quantize<T>(xv, p, a.inv2e, a.twoe, a.el, a.R, xr);
      gmem(f.code[d])[fi] = (uint16_t)q;  // d is the point's lowest family
      face_store<T>(f, a.g, x, xr);
    } else {
      const uint32_t q = (d == 2 && E.fcode2) ? (uint32_t)gmem(f.code[2])[fi]
                                              : (uint32_t)code[brick_pos(a.g.n, x)];
      const T v = q ? recon<T>(p, (double)((int32_t)q - (int32_t)a.R), a.twoe) : out[idx];
      face_store<T>(f, a.g, x, v);
    }
  }
}

// ---------------------------------------------------------------------------
// Coarse face levels on whole planes.  A point of a face plane is predicted from
// points of the same plane (its odd dims lie in the plane), so a plane is a 2D
// problem; its levels s >= 4 use only the plane's lattice (every 4th point
// along active dims), which for planes up to a few hundred points per side
// fits one work-group's LDS.  The plane box spans the whole plane, so the
// stencils' ends are the field's ends as in the face steps.  Points on lines
// shared with a lower family are computed in both planes (same neighbours,
// same values); each plane writes its own family's face array, and codes only
// of the points whose lowest family it is.

// n / d with a host-computed exact multiplier (shift -1: d <= 1)
__device__ __forceinline__ uint32_t div_magic(uint32_t n, uint32_t m, int32_t sh)
{
  return xdiv(n, XDivisor{m, sh});
}

template <typename T>
struct PlaneCompressOp {
  using Fetched = int;
  T* L;
  const FaceGeo* f;
  const Geom* g;
  int32_t d;
  int64_t xd;  // the plane's coordinate along d
  int32_t k0, k1, k2;
  uint32_t R;
  double el, inv2e, twoe;
  __device__ __forceinline__ int fetch(int32_t, int32_t, int32_t, bool) const { return 0; }
  __device__ __forceinline__ void apply(int32_t li, int32_t x0, int32_t x1, int32_t x2, T p, int)
  {
    const T xv = L[li];
    T xr = xv;
    const uint32_t q = quantize<T>(xv, p, inv2e, twoe, el, R, xr);
    L[li] = xr;
    int64_t x[4] = {(int64_t)x0 * k0, (int64_t)x1 * k1, (int64_t)x2 * k2, 0};
    x[d] = xd;
    if (low_family(*f, *g, x) == d) gmem(f->code[d])[face_index(*f, d, x)] = (uint16_t)q;
  }
};

template <typename T>
struct PlaneDecompressOp {
  using Fetched = uint32_t;
  T* L;
  const Geom* g;
  const HPEZ_GLOBAL uint16_t* code;
  const HPEZ_GLOBAL T* out;
  int32_t d;
  int64_t xd;
  int32_t k0, k1, k2;
  uint32_t R;
  double twoe;
  __device__ __forceinline__ void pos(int32_t x0, int32_t x1, int32_t x2, int64_t* x) const
  {
    x[0] = (int64_t)x0 * k0;
    x[1] = (int64_t)x1 * k1;
    x[2] = (int64_t)x2 * k2;
    x[3] = 0;
    x[d] = xd;
  }
  __device__ __forceinline__ uint32_t fetch(int32_t x0, int32_t x1, int32_t x2, bool ok) const
  {
    if (!ok) return 0u;
    int64_t x[4];
    pos(x0, x1, x2, x);
    return (uint32_t)code[brick_pos(g->n, x)];
  }
  __device__ __forceinline__ void apply(int32_t li, int32_t x0, int32_t x1, int32_t x2, T p, uint32_t q)
  {
    if (q) {
      L[li] = recon<T>(p, (double)((int32_t)q - (int32_t)R), twoe);
    } else {
      int64_t x[4];
      pos(x0, x1, x2, x);
      L[li] = out[x[0] * g->st[0] + x[1] * g->st[1] + x[2] * g->st[2] + x[3]];
    }
  }
};

template <typename T, int MODE>
__global__ void __launch_bounds__(kBlockThreads) plane_kernel(const PlaneJob<T>* __restrict__ tab,
                                                              const uint64_t* __restrict__ wg_begin,
                                                              int n)
{
  constexpr int NT = kBlockThreads;
  extern __shared__ unsigned char lds_raw[];
  T* L = reinterpret_cast<T*>(lds_raw);
  const int j = find_entry(wg_begin, n, blockIdx.x);
  const PlaneJob<T>& J = tab[j];
  const Geom& g = J.g;
  const FaceGeo& f = J.f;
  const int32_t d = J.d;
  const int64_t xd = (int64_t)(blockIdx.x - J.wg_begin) << f.blog2;
  Box lb;
  lb.E0 = J.E[0];
  lb.E1 = J.E[1];
  lb.E2 = J.E[2];
  lb.b1 = lb.E2;
  lb.b0 = lb.E1 * lb.E2;
  lb.a0 = d != 0 && g.act[0];
  lb.a1 = d != 1 && g.act[1];
  lb.a2 = d != 2 && g.act[2];
  lb.lo0 = lb.lo1 = lb.lo2 = 0;
  lb.hi0 = lb.E0 - 1;
  lb.hi1 = lb.E1 - 1;
  lb.hi2 = lb.E2 - 1;
  const int32_t k0 = lb.a0 ? 4 : 1, k1 = lb.a1 ? 4 : 1, k2 = lb.a2 ? 4 : 1;
  const uint32_t ncell = (uint32_t)(lb.E0 * lb.b0);
  const HPEZ_GLOBAL T* F = gmem(reinterpret_cast<const T*>(f.val[d]));
  const HPEZ_GLOBAL T* X = gmem(J.X);
  // the lattice: points of the coarse grid (multiples of B) from the face
  // array, the others from X (compress) or predicted (decompress)
  // (a lane's loads are all issued before the first of them is waited for)
  constexpr int UC = 8;
  for (uint32_t ib = 0; ib < ncell; ib += UC * NT) {
    T v[UC];
#pragma unroll
    for (int u = 0; u < UC; u++) {
      const uint32_t i = ib + u * NT + threadIdx.x;
      const uint32_t ii = i < ncell ? i : 0u;
      const uint32_t q0 = div_magic(ii, J.mg_b0, J.sh_b0);
      const uint32_t r = ii - q0 * (uint32_t)lb.b0;
      const uint32_t q1 = div_magic(r, J.mg_e2, J.sh_e2);
      int64_t x[4] = {(int64_t)q0 * k0, (int64_t)q1 * k1, (int64_t)(r - q1 * (uint32_t)lb.E2) * k2,
                      0};
      x[d] = xd;
      bool grid = true;
      for (int e = 0; e < 3; e++)
        if (g.act[e] && (x[e] & (f.B - 1))) grid = false;
      const HPEZ_GLOBAL T* src = grid ? F + face_index(f, d, x)
                                      : X + (x[0] * g.st[0] + x[1] * g.st[1] + x[2] * g.st[2] + x[3]);
      const bool ok = i < ncell && (grid || MODE == 0);
      v[u] = ok ? *src : (T)0;
    }
#pragma unroll
    for (int u = 0; u < UC; u++) {
      const uint32_t i = ib + u * NT + threadIdx.x;
      if (i < ncell) L[i] = v[u];
    }
  }
  __syncthreads();
  for (int l = J.Ltop; l > kCoarseL; l--) {
    const int32_t s = 1 << (l - 1 - 2);  // lattice stride
    const hpez_interp& c = J.level[l - 1];
    if (MODE == 0) {
      PlaneCompressOp<T> op{L,  &f, &g, d, xd, k0, k1, k2, J.R, J.el_l[l], J.inv2e_l[l],
                            J.twoe_l[l]};
      box_level<T, NT>(c, lb, L, 0, 0, 0, s, J.wmd, op);
    } else {
      PlaneDecompressOp<T> op{L, &g, gmem(J.code), gmem(J.out), d, xd, k0, k1, k2, J.R, J.twoe_l[l]};
      box_level<T, NT>(c, lb, L, 0, 0, 0, s, J.wmd, op);
    }
  }
  HPEZ_GLOBAL T* Fw = gmem(reinterpret_cast<T*>(f.val[d]));
  for (uint32_t i = threadIdx.x; i < ncell; i += NT) {
    const uint32_t q0 = div_magic(i, J.mg_b0, J.sh_b0);
    const uint32_t r = i - q0 * (uint32_t)lb.b0;
    const uint32_t q1 = div_magic(r, J.mg_e2, J.sh_e2);
    int64_t x[4] = {(int64_t)q0 * k0, (int64_t)q1 * k1, (int64_t)(r - q1 * (uint32_t)lb.E2) * k2, 0};
    x[d] = xd;
    Fw[face_index(f, d, x)] = L[i];
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

// four consecutive values; p is 16-byte aligned
template <typename T>
struct Quad {
  T v[4];
};
// plain vector types (no class constructors, so loads and stores work through
// address-space qualified pointers)
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef double vd2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ Quad<float> load_quad(const HPEZ_GLOBAL float* p)
{
  const vf4 q = *reinterpret_cast<const HPEZ_GLOBAL vf4*>(p);
  return {{q.x, q.y, q.z, q.w}};
}
__device__ __forceinline__ Quad<double> load_quad(const HPEZ_GLOBAL double* p)
{
  const vd2 a = reinterpret_cast<const HPEZ_GLOBAL vd2*>(p)[0];
  const vd2 b = reinterpret_cast<const HPEZ_GLOBAL vd2*>(p)[1];
  return {{a.x, a.y, b.x, b.y}};
}
// the same with the streaming hint: the field is read once, and its lines
// should leave the cache before the partly written code lines do
__device__ __forceinline__ Quad<float> load_quad_once(const HPEZ_GLOBAL float* p)
{
  const vf4 q = __builtin_nontemporal_load(reinterpret_cast<const HPEZ_GLOBAL vf4*>(p));
  return {{q.x, q.y, q.z, q.w}};
}
__device__ __forceinline__ Quad<double> load_quad_once(const HPEZ_GLOBAL double* p)
{
  const vd2 a = __builtin_nontemporal_load(reinterpret_cast<const HPEZ_GLOBAL vd2*>(p));
  const vd2 b = __builtin_nontemporal_load(reinterpret_cast<const HPEZ_GLOBAL vd2*>(p) + 1);
  return {{a.x, a.y, b.x, b.y}};
}

// per-point work of the compress schedule: quantize, emit the code, write the
// reconstruction back, count the code
template <typename T>
struct CompressOp {
  using Fetched = int;
  T* L;
  HPEZ_GLOBAL uint16_t* code;  // the brick's codes
  uint32_t* lh;
  HPEZ_GLOBAL uint32_t* hist;
  int32_t Eb1, Eb2;
  uint32_t R, lo;
  double el, inv2e, twoe;
  uint32_t nR;  // codes equal to R (zero residual), counted per lane
  __device__ __forceinline__ int fetch(int32_t, int32_t, int32_t, bool) const { return 0; }
  __device__ __forceinline__ void apply(int32_t li, int32_t x0, int32_t x1, int32_t x2, T p, int)
  {
    const T xv = L[li];
    T xr = xv;
    const uint32_t q = quantize<T>(xv, p, inv2e, twoe, el, R, xr);
    code[(uint32_t)((x0 * Eb1 + x1) * Eb2 + x2)] = (uint16_t)q;
    L[li] = xr;
    // the most frequent code is counted in a register, the others in LDS
    nR += q == R;
    if (q != R) {
      // distinct scopes keep the LDS and the global update apart (no generic pointer)
      const uint32_t w = q - lo;
      if (w < (uint32_t)kBlockHistWin)
        __hip_atomic_fetch_add(&lh[w], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      else
        __hip_atomic_fetch_add(&hist[q], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
};

// per-point work of the decompress schedule: the code is fetched first, then
// x' = p + q 2e_l, or the stored value for code 0
template <typename T>
struct DecompressOp {
  using Fetched = uint32_t;
  T* L;
  const HPEZ_GLOBAL uint16_t* code;  // the brick's codes
  const HPEZ_GLOBAL T* out;
  int64_t o0, o1, o2, st0, st1;
  int32_t Eb1, Eb2;
  uint32_t R;
  double twoe;
  __device__ __forceinline__ uint32_t fetch(int32_t x0, int32_t x1, int32_t x2, bool ok) const
  {
    return ok ? (uint32_t)code[(uint32_t)((x0 * Eb1 + x1) * Eb2 + x2)] : 0u;
  }
  __device__ __forceinline__ void apply(int32_t li, int32_t x0, int32_t x1, int32_t x2, T p, uint32_t q)
  {
    L[li] = q ? recon<T>(p, (double)((int32_t)q - (int32_t)R), twoe)
              : out[(o0 + x0) * st0 + (o1 + x1) * st1 + (o2 + x2)];
  }
};

// ---------------------------------------------------------------------------
// Coarse levels of the blocks (s >= kCoarseS) on each block's lattice: the box
// cells whose coordinates are multiples of 4 along every active dim (all cells
// along an inactive one).  In lattice coordinates (cell / 4 on active dims) a
// level of stride s is a level of stride s / 4 with the same neighbours and the
// same boundary ladder (last = floor((E - 1) / 4)), so the box schedule runs on
// the lattice unchanged.  A block's lattice is small (at most 9 x 9 x 32
// cells), so one wave takes a block and many blocks share a CU; the block
// kernel then starts at level kCoarseL.  Output per block: the lattice values
// (reconstructed) and, compressing, the codes of the lattice points.

// lattice cells of a box: active dims (E - 1) / 4 + 1, inactive dims E
__device__ __forceinline__ void lattice_box(const Box& bx, Box& lb)
{
  lb.E0 = bx.a0 ? (bx.E0 - 1) / 4 + 1 : bx.E0;
  lb.E1 = bx.a1 ? (bx.E1 - 1) / 4 + 1 : bx.E1;
  lb.E2 = bx.a2 ? (bx.E2 - 1) / 4 + 1 : bx.E2;
  lb.b1 = lb.E2;
  lb.b0 = lb.E1 * lb.E2;
  lb.a0 = bx.a0;
  lb.a1 = bx.a1;
  lb.a2 = bx.a2;
  lb.lo0 = bx.lo0;
  lb.lo1 = bx.lo1;
  lb.lo2 = bx.lo2;
  lb.hi0 = bx.a0 ? bx.hi0 / 4 : bx.hi0;
  lb.hi1 = bx.a1 ? bx.hi1 / 4 : bx.hi1;
  lb.hi2 = bx.a2 ? bx.hi2 / 4 : bx.hi2;
}

template <typename T>
struct CoarseCompressOp {
  using Fetched = int;
  T* L;
  HPEZ_GLOBAL uint16_t* ccode;  // the block's lattice codes, lattice order
  uint32_t R;
  double el, inv2e, twoe;
  __device__ __forceinline__ int fetch(int32_t, int32_t, int32_t, bool) const { return 0; }
  __device__ __forceinline__ void apply(int32_t li, int32_t, int32_t, int32_t, T p, int)
  {
    const T xv = L[li];
    T xr = xv;
    const uint32_t q = quantize<T>(xv, p, inv2e, twoe, el, R, xr);
    ccode[li] = (uint16_t)q;
    L[li] = xr;
  }
};

template <typename T>
struct CoarseDecompressOp {
  using Fetched = uint32_t;
  T* L;
  const HPEZ_GLOBAL uint16_t* code;  // the brick's codes
  const HPEZ_GLOBAL T* out;
  int64_t o0, o1, o2, st0, st1;
  int32_t Eb1, Eb2;
  int32_t k0, k1, k2;  // cells per lattice step (4 active, 1 inactive)
  uint32_t R;
  double twoe;
  __device__ __forceinline__ uint32_t fetch(int32_t x0, int32_t x1, int32_t x2, bool ok) const
  {
    return ok ? (uint32_t)code[(uint32_t)((x0 * k0 * Eb1 + x1 * k1) * Eb2 + x2 * k2)] : 0u;
  }
  __device__ __forceinline__ void apply(int32_t li, int32_t x0, int32_t x1, int32_t x2, T p, uint32_t q)
  {
    L[li] = q ? recon<T>(p, (double)((int32_t)q - (int32_t)R), twoe)
              : out[(o0 + x0 * k0) * st0 + (o1 + x1 * k1) * st1 + (o2 + x2 * k2)];
  }
};

template <typename T, int MODE>
__global__ void __launch_bounds__(64) coarse_kernel(const BlockJobDev<T>* __restrict__ jobs,
                                                    const uint64_t* __restrict__ begin, int njobs)
{
  __shared__ T L[kCoarseCells];
  const uint64_t gbi = blockIdx.x;
  const int jb = find_entry(begin, njobs, gbi);
  const BlockJobDev<T>& J = jobs[jb];
  const BlockArgs& a = J.a;
  const FaceGeo& f = J.f;
  const uint64_t bi = gbi - begin[jb];
  Block3 bk;
  Box bx, lb;
  block_geometry(a.g, (int64_t)bi, a.nb, bk, bx);
  lattice_box(bx, lb);
  const int32_t k0 = bx.a0 ? 4 : 1, k1 = bx.a1 ? 4 : 1, k2 = bx.a2 ? 4 : 1;
  const uint32_t n = (uint32_t)(lb.E0 * lb.b0);
  const Divisor mb0 = fmagic((uint32_t)lb.b0), mE2 = fmagic((uint32_t)lb.E2);
  const int64_t st0 = a.g.st[0], st1 = a.g.st[1];
  const HPEZ_GLOBAL T* __restrict__ X = gmem(J.X);
  // the lattice: face cells from the face arrays, the others from X (compress);
  // a lane's loads are all issued before the first of them is waited for
  constexpr int UC = 12;
  for (uint32_t ib = 0; ib < n; ib += UC * 64) {
    T v[UC];
#pragma unroll
    for (int u = 0; u < UC; u++) {
      const uint32_t i = ib + u * 64 + threadIdx.x;
      const uint32_t ii = i < n ? i : 0u;
      const uint32_t q0 = fdiv(ii, mb0);
      const uint32_t r = ii - q0 * (uint32_t)lb.b0;
      const uint32_t q1 = fdiv(r, mE2);
      const int32_t c0 = (int32_t)q0 * k0, c1 = (int32_t)q1 * k1,
                    c2 = (int32_t)(r - q1 * (uint32_t)lb.E2) * k2;
      const int64_t x0 = bk.o0 + c0, x1 = bk.o1 + c1, x2 = bk.o2 + c2;
      const HPEZ_GLOBAL T* src = X + (x0 * st0 + x1 * st1 + x2);
      bool ok = i < n && MODE == 0;
      if (bx.a0 && (c0 == 0 || c0 == kBrick)) {
        src = gmem(reinterpret_cast<const T*>(f.val[0])) + ((x0 >> f.blog2) * f.plane[0] +
                                                            x1 * f.fs[0][1] + x2);
        ok = i < n;
      } else if (bx.a1 && (c1 == 0 || c1 == kBrick)) {
        src = gmem(reinterpret_cast<const T*>(f.val[1])) + ((x1 >> f.blog2) * f.plane[1] +
                                                            x0 * f.fs[1][0] + x2);
        ok = i < n;
      } else if (bx.a2 && (c2 == 0 || c2 == kBrick)) {
        src = gmem(reinterpret_cast<const T*>(f.val[2])) + ((x2 >> f.blog2) * f.plane[2] +
                                                            x0 * f.fs[2][0] + x1 * f.fs[2][1]);
        ok = i < n;
      }
      v[u] = ok ? *src : (T)0;
    }
#pragma unroll
    for (int u = 0; u < UC; u++) {
      const uint32_t i = ib + u * 64 + threadIdx.x;
      if (i < n) L[i] = v[u];
    }
  }
  __syncthreads();
  const hpez_interp c = a.cand[gmem(J.bcfg)[bi]];
  const int64_t p0 = bk.o0 / k0, p1 = bk.o1 / k1, p2 = bk.o2 / k2;  // lattice origin
  const uint64_t brick_base = (uint64_t)(bk.o0 * a.g.n[1] * a.g.n[2] +
                                         bk.Eb0 * bk.o1 * a.g.n[2] + bk.Eb0 * bk.Eb1 * bk.o2);
  for (int l = a.L; l > kCoarseL; l--) {
    const int32_t s = 1 << (l - 1 - 2);  // lattice stride
    if (MODE == 0) {
      CoarseCompressOp<T> op{L, gmem(J.ccode) + bi * kCoarseCells, a.R, a.el_l[l], a.inv2e_l[l],
                             a.twoe_l[l]};
      box_level<T, 64>(c, lb, L, p0, p1, p2, s, a.wmd, op);
    } else {
      CoarseDecompressOp<T> op{L,  gmem(J.code) + brick_base, gmem(J.out), bk.o0, bk.o1, bk.o2,
                               st0, st1, bk.Eb1, bk.Eb2, k0, k1, k2, a.R, a.twoe_l[l]};
      box_level<T, 64>(c, lb, L, p0, p1, p2, s, a.wmd, op);
    }
  }
  HPEZ_GLOBAL T* cv = gmem(J.cval) + bi * kCoarseCells;
  for (uint32_t i = threadIdx.x; i < n; i += 64) cv[i] = L[i];
}

// Box loading: rows along dim 2 in quads of four cells.  Face rows (c0 or c1
// on a block face) come from the face arrays, cells c2 = 0 / 32 from the dim-2
// faces, everything else from X (compress only).  Item `it` of a block is row
// it / nq, quad it % nq.
struct BoxItems {
  int32_t E1, E2, nq;
  uint32_t rowq, nitems;
  Divisor mgr, mgq;
};

__device__ __forceinline__ BoxItems box_items(const Box& bx)
{
  BoxItems b;
  b.E1 = bx.E1;
  b.E2 = bx.E2;
  b.nq = (bx.E2 + 3) >> 2;
  b.rowq = (uint32_t)(bx.E1 * b.nq);
  b.nitems = (uint32_t)bx.E0 * b.rowq;
  b.mgr = fmagic(b.rowq);
  b.mgq = fmagic((uint32_t)b.nq);
  return b;
}

// Where item `it` of a box goes: its cells (box row c0, c1, cells cb .. cb +
// cnt - 1 along dim 2), their LDS base, and which of them are loaded (wr):
// face cells from the face arrays, interior cells from the field (compress,
// cell 32 excluded: the next block's face) or from the codes (decompressing
// a full block), and the row's dim-2 face cell.
struct ItemPos {
  int32_t c0, c1, cb, cnt;
  int32_t lbase;
  uint32_t wr;
  bool face0, face1, face2;
};

template <int MODE>
__device__ __forceinline__ ItemPos item_pos(const Box& bx, const BoxItems& bi, uint32_t it, bool fast)
{
  ItemPos p;
  p.wr = 0;
  p.lbase = 0;
  p.c0 = p.c1 = p.cb = p.cnt = 0;
  p.face0 = p.face1 = p.face2 = false;
  if (it >= bi.nitems) return p;
  p.c0 = (int32_t)fdiv(it, bi.mgr);
  const uint32_t rr = it - (uint32_t)p.c0 * bi.rowq;
  p.c1 = (int32_t)fdiv(rr, bi.mgq);
  p.cb = 4 * (int32_t)(rr - (uint32_t)p.c1 * bi.nq);
  p.cnt = bi.E2 - p.cb < 4 ? bi.E2 - p.cb : 4;
  // row-major box, or the parity-split slots of a full block (cb even)
  p.lbase = fast ? fslot(p.c0) * kFP0 + fslot(p.c1) * kFP1 + (p.cb >> 1)
                 : (p.c0 * bi.E1 + p.c1) * bi.E2 + p.cb;
  p.face0 = bx.a0 && (p.c0 == 0 || p.c0 == kBrick);
  p.face1 = !p.face0 && bx.a1 && (p.c1 == 0 || p.c1 == kBrick);
  p.face2 = !p.face0 && !p.face1 && bx.a2 && (p.cb == 0 || p.cb == kBrick);
  const bool interior = !p.face0 && !p.face1 && p.cb < kBrick;
  if (p.face0 || p.face1 || (MODE == 0 && interior)) p.wr = (1u << p.cnt) - 1u;
  else if (MODE == 1 && fast && interior) p.wr = 0xFu;
  if (p.face2) p.wr |= 1u;
  return p;
}

// the values of one item (cnt <= 4 cells; the cells item_pos marks) and, in
// pos, its LDS base (below 33^3 < 2^16) with the loaded-cell mask at bit 16:
// one register per item held until the store
template <typename T, int MODE>
__device__ __forceinline__ Quad<T> load_item(const FaceGeo& f, const HPEZ_GLOBAL T* __restrict__ X, int64_t st0,
                                             int64_t st1, const Block3& bk, const Box& bx,
                                             const BoxItems& bi, uint32_t it, bool vec,
                                             bool fast, const HPEZ_GLOBAL uint16_t* bcode,
                                             uint32_t& pos)
{
  Quad<T> v;
#pragma unroll
  for (int j = 0; j < 4; j++) v.v[j] = (T)0;
  const ItemPos p = item_pos<MODE>(bx, bi, it, fast);
  pos = (uint32_t)p.lbase | p.wr << 16;
  if (!p.wr) return v;
  const int32_t c0 = p.c0, c1 = p.c1, cb = p.cb, cnt = p.cnt;
  const int64_t x0 = bk.o0 + c0, x1 = bk.o1 + c1, x2 = bk.o2 + cb;
  const bool face0 = p.face0, face1 = p.face1;
  const HPEZ_GLOBAL T* src = nullptr;
  bool once = false;
  if (face0)
    src = gmem(reinterpret_cast<const T*>(f.val[0])) + (x0 >> f.blog2) * f.plane[0] + x1 * f.fs[0][1] + x2;
  else if (face1)
    src = gmem(reinterpret_cast<const T*>(f.val[1])) + (x1 >> f.blog2) * f.plane[1] + x0 * f.fs[1][0] + x2;
  else if (MODE == 0 && cb < kBrick) {
    src = X + x0 * st0 + x1 * st1 + x2;  // (cell c2 = 32 is the next block's face value)
    once = true;
  }
  if (MODE == 1 && fast && !src && cb < kBrick) {
    // decompressing a full block: the interior rows' cells take the points'
    // codes (as raw bits) until the points are reconstructed
    const uint64_t cw =
        *reinterpret_cast<const HPEZ_GLOBAL uint64_t*>(bcode + (c0 * kBrick + c1) * kBrick + cb);
#pragma unroll
    for (int j = 0; j < 4; j++) v.v[j] = (T)__uint_as_float((uint32_t)(cw >> (16 * j)) & 0xFFFFu);
  }
  if (src) {
    if (vec && cnt == 4 && once) {
      v = load_quad_once(src);
    } else if (vec && cnt == 4) {
      v = load_quad(src);
    } else {
#pragma unroll
      for (int j = 0; j < 4; j++)
        if (j < cnt) v.v[j] = src[j];
    }
  }
  if (p.face2) {
    // the row's cell on a dim-2 face
    v.v[0] = gmem(reinterpret_cast<const T*>(f.val[2]))[(x2 >> f.blog2) * f.plane[2] +
                                                        x0 * f.fs[2][0] + x1 * f.fs[2][1]];
  }
  return v;
}

template <typename T>
__device__ __forceinline__ void store_item(T* L, const Quad<T>& v, uint32_t pos, bool fast)
{
  // pos as load_item gives it
  const int32_t lbase = (int32_t)(pos & 0xFFFFu);
  const uint32_t wr = pos >> 16;
  // full blocks: cells cb, cb + 2 at even slots cb / 2, cb / 2 + 1; cb + 1, cb + 3
  // at odd slots 17 + cb / 2, 18 + cb / 2
#pragma unroll
  for (int j = 0; j < 4; j++)
    if (wr >> j & 1u) L[lbase + (fast ? (j >> 1) + 17 * (j & 1) : j)] = v.v[j];
}

// stream position of a brick's first point (all earlier bricks are full along
// the dims before the last partial one)
__device__ __forceinline__ uint64_t brick_start(const Geom& g, const Block3& bk)
{
  return (uint64_t)(bk.o0 * g.n[1] * g.n[2] + bk.Eb0 * bk.o1 * g.n[2] + bk.Eb0 * bk.Eb1 * bk.o2);
}

// a block whose levels below the lattice take the full-block schedule: a
// 32^3 brick with all dims active whose configuration is not
// multi-dimensional same-level cubic (those take the row-major box)
__device__ __forceinline__ bool full_block(const Block3& bk, const Box& bx, const hpez_interp& c)
{
  return bx.a0 && bx.a1 && bx.a2 && bk.Eb0 == kBrick && bk.Eb1 == kBrick && bk.Eb2 == kBrick &&
         !(c.md && c.same_level && c.kind != 0);
}

// the LDS histogram window of job J into its histogram
template <typename T>
__device__ __forceinline__ void hist_flush(const uint32_t* lh, const BlockJobDev<T>& J, int nt)
{
  HPEZ_GLOBAL uint32_t* hist = gmem(J.hist);
  const uint32_t lo = J.a.hist_lo;
  for (int i = threadIdx.x; i < kBlockHistWin; i += nt)
    if (lh[i]) __hip_atomic_fetch_add(&hist[lo + i], lh[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Persistent work-groups (one per CU): blocks are taken from a counter; for
// float boxes the next block's loads are issued before the current block's
// levels, so they complete while it computes.
// NT = kBlockThreads: any box, one work-group per CU.  NT = kSmallBoxThreads:
// only boxes of at most two active dims and 33 x 33 points or fewer (so at
// most 33 x 33 load items and 2 x 32 face codes), several work-groups per CU;
// the full-block schedule (three active dims) is not compiled in.
template <typename T, int MODE, int NT>
__global__ void __launch_bounds__(NT, NT == kBlockThreads ? 1 : 4) block_kernel(const BlockJobDev<T>* __restrict__ jobs,
                                                              const uint64_t* __restrict__ begin,
                                                              int njobs,
                                                              uint32_t lh_off)
{
  constexpr bool FULL = NT == kBlockThreads;  // full blocks (33^3 slot layout) possible
  constexpr bool PREF = sizeof(T) == 4;
  // items per lane held across a block
  constexpr int UP = PREF ? ((FULL ? 33 * 33 * 9 : 33 * 33) + NT - 1) / NT : 1;
  extern __shared__ unsigned char lds_raw[];
  T* L = reinterpret_cast<T*>(lds_raw);
  const uint64_t nbt = begin[njobs];
  // compress: the LDS histogram window sits after the largest box of the
  // launch and accumulates every block of one job the work-group takes;
  // its counts reach the job's histogram when the work-group moves to
  // another job or ends (one flush per work-group instead of one per block)
  uint32_t* lh = reinterpret_cast<uint32_t*>(lds_raw + lh_off);
  int hjob = -1;

  // blocks are dealt round-robin: work-group w takes w, w + G, w + 2G, ...
  // (G work-groups; blocks cost about the same, and no counter round trip
  // stands between two blocks)
  uint64_t gbi = blockIdx.x;
  Quad<T> pv[UP];
  uint32_t ppos[UP];
  T pcv = (T)0;  // the lane's first lattice value of the next block
  if (PREF && gbi < nbt) {
    const int j = find_entry(begin, njobs, gbi);
    const BlockJobDev<T>& J = jobs[j];
    Block3 bk;
    Box bx;
    block_geometry(J.a.g, (int64_t)(gbi - begin[j]), J.a.nb, bk, bx);
    const BoxItems its = box_items(bx);
    const bool fast1 = FULL && full_block(bk, bx, J.a.cand[gmem(J.bcfg)[gbi - begin[j]]]);
#pragma unroll
    for (int u = 0; u < UP; u++)
      pv[u] = load_item<T, MODE>(J.f, gmem(J.X), J.a.g.st[0], J.a.g.st[1], bk, bx, its,
                                 threadIdx.x + u * NT, J.a.vec != 0, fast1,
                                 gmem(J.code) + brick_start(J.a.g, bk), ppos[u]);
    Box lb1;
    lattice_box(bx, lb1);
    if (threadIdx.x < (uint32_t)(lb1.E0 * lb1.b0))
      pcv = gmem(J.cval)[(gbi - begin[j]) * kCoarseCells + threadIdx.x];
  }

  while (gbi < nbt) {
    __syncthreads();  // the previous block is done with LDS
    const int jb = find_entry(begin, njobs, gbi);
    const BlockJobDev<T>& J = jobs[jb];
    const BlockArgs& a = J.a;
    const FaceGeo& f = J.f;
    const HPEZ_GLOBAL T* __restrict__ X = gmem(J.X);
    HPEZ_GLOBAL uint16_t* __restrict__ code = gmem(J.code);
    HPEZ_GLOBAL uint32_t* __restrict__ hist = gmem(J.hist);
    HPEZ_GLOBAL T* __restrict__ out = gmem(J.out);
    const uint64_t bi = gbi - begin[jb];
    const int64_t st0 = a.g.st[0], st1 = a.g.st[1];
    const uint32_t lo = a.hist_lo;
    // rows are 16-byte aligned in X, out and the face arrays (host-checked)
    const bool vec = a.vec != 0;
    Block3 bk;
    Box bx;
    block_geometry(a.g, (int64_t)bi, a.nb, bk, bx);
    const bool fast = FULL && PREF && full_block(bk, bx, a.cand[gmem(J.bcfg)[bi]]);
    // stream position of the brick's first point (all earlier bricks are full
    // along the dims before the last partial one)
    const uint64_t brick_base = brick_start(a.g, bk);
    // a full block's slots span 33 per dim whatever its box extents
    const uint32_t nbox = fast ? (uint32_t)(33 * kFP0) : (uint32_t)bx.E0 * bx.b0;  // <= lh_off / sizeof(T)
    (void)nbox;
    const int32_t E1 = bx.E1, E2 = bx.E2, Eb1 = bk.Eb1, Eb2 = bk.Eb2;
    if (MODE == 0 && jb != hjob) {
      // the window holds another job's counts: flush them (each lane its own
      // entries, so no barrier between the flush and the clear)
      if (hjob >= 0) hist_flush(lh, jobs[hjob], NT);
      for (uint32_t i = threadIdx.x; i < (uint32_t)kBlockHistWin; i += NT) lh[i] = 0;
      hjob = jb;
    }
    // ---- the box into LDS
    if (PREF) {
#pragma unroll
      for (int u = 0; u < UP; u++) store_item<T>(L, pv[u], ppos[u], fast);
    } else {
      const BoxItems its = box_items(bx);
      constexpr int UL = 4;
      for (uint32_t ib = threadIdx.x; ib < its.nitems; ib += UL * NT) {
        Quad<T> v[UL];
        uint32_t pos[UL];
#pragma unroll
        for (int u = 0; u < UL; u++)
          v[u] = load_item<T, MODE>(f, X, st0, st1, bk, bx, its, ib + u * NT, vec, false, nullptr,
                                    pos[u]);
#pragma unroll
        for (int u = 0; u < UL; u++) store_item<T>(L, v[u], pos[u], false);
      }
    }
    // the lattice cells hold the coarse levels' results
    __syncthreads();
    Box lb;
    lattice_box(bx, lb);
    const int32_t lk0 = bx.a0 ? 4 : 1, lk1 = bx.a1 ? 4 : 1, lk2 = bx.a2 ? 4 : 1;
    const uint32_t nlat = (uint32_t)(lb.E0 * lb.b0);
    const Divisor mlb0 = fmagic((uint32_t)lb.b0), mlE2 = fmagic((uint32_t)lb.E2);
    {
      const HPEZ_GLOBAL T* cv = gmem(J.cval) + bi * kCoarseCells;
      for (uint32_t i = threadIdx.x; i < nlat; i += NT) {
        const uint32_t q0 = fdiv(i, mlb0);
        const uint32_t r = i - q0 * (uint32_t)lb.b0;
        const uint32_t q1 = fdiv(r, mlE2);
        const uint32_t q2 = r - q1 * (uint32_t)lb.E2;
        T v;
        if (PREF && i == threadIdx.x) v = pcv;  // prefetched with the box
        else v = cv[i];
        L[fast ? 2 * ((int32_t)q0 * kFP0 + (int32_t)q1 * kFP1 + (int32_t)q2)
               : ((int32_t)q0 * lk0 * E1 + (int32_t)q1 * lk1) * E2 + (int32_t)q2 * lk2] = v;
      }
    }
    // compress: the codes of the brick's own faces (c_d = 0 on an active dim)
    // from the face code arrays; loaded now, stored and counted after the
    // levels, so the loads complete while the block computes
    // face codes per lane: 3 x 32 x 32 <= 3 NT for any box; a box of at most two
    // active dims has at most 2 x 32 face codes (<= NT)
    constexpr int FC = MODE == 0 ? (FULL ? 3 : 1) : 1;
    uint32_t fcv[FC], fcd[FC];
    bool fok[FC];
    if (MODE == 0) {
      const int32_t Eb0 = bk.Eb0;
      const int32_t r0 = bx.a0, r1 = bx.a1;
      const int32_t f0n = bx.a0 ? Eb1 * Eb2 : 0;
      const int32_t f1n = bx.a1 ? (Eb0 - r0) * Eb2 : 0;
      const int32_t f2n = bx.a2 ? (Eb0 - r0) * (Eb1 - r1) : 0;
      const Divisor dE2 = fmagic((uint32_t)Eb2);
      const Divisor dE1 = fmagic((uint32_t)(Eb1 - r1 > 0 ? Eb1 - r1 : 1));
#pragma unroll
      for (int u = 0; u < FC; u++) {
        const int32_t j = (int32_t)threadIdx.x + u * NT;
        fok[u] = j < f0n + f1n + f2n;
        fcv[u] = 0;
        fcd[u] = 0;
        if (!fok[u]) continue;
        if (j < f0n) {
          const int32_t c1 = (int32_t)fdiv((uint32_t)j, dE2), c2 = j - c1 * Eb2;
          fcd[u] = (uint32_t)(c1 * Eb2 + c2);
          fcv[u] = gmem(f.code[0])[(bk.o0 >> f.blog2) * f.plane[0] + (bk.o1 + c1) * f.fs[0][1] +
                             (bk.o2 + c2) * f.fs[0][2]];
        } else if (j < f0n + f1n) {
          const int32_t jj = j - f0n;
          const int32_t q = (int32_t)fdiv((uint32_t)jj, dE2);
          const int32_t c0 = r0 + q, c2 = jj - q * Eb2;
          fcd[u] = (uint32_t)(c0 * Eb1 * Eb2 + c2);
          fcv[u] = gmem(f.code[1])[(bk.o1 >> f.blog2) * f.plane[1] + (bk.o0 + c0) * f.fs[1][0] +
                             (bk.o2 + c2) * f.fs[1][2]];
        } else {
          const int32_t jj = j - f0n - f1n;
          const int32_t q = (int32_t)fdiv((uint32_t)jj, dE1);
          const int32_t c0 = r0 + q, c1 = r1 + (jj - q * (Eb1 - r1));
          fcd[u] = (uint32_t)((c0 * Eb1 + c1) * Eb2);
          fcv[u] = gmem(f.code[2])[(bk.o2 >> f.blog2) * f.plane[2] + (bk.o0 + c0) * f.fs[2][0] +
                             (bk.o1 + c1) * f.fs[2][1]];
        }
      }
    }
    __syncthreads();
    const uint64_t bn = gbi + gridDim.x;
    if (PREF && bn < nbt) {
      // the next block's loads, in flight during this block's levels
      const int j2 = find_entry(begin, njobs, bn);
      const BlockJobDev<T>& J2 = jobs[j2];
      Block3 bk2;
      Box bx2;
      block_geometry(J2.a.g, (int64_t)(bn - begin[j2]), J2.a.nb, bk2, bx2);
      const BoxItems its2 = box_items(bx2);
      const bool fast2 = FULL && full_block(bk2, bx2, J2.a.cand[gmem(J2.bcfg)[bn - begin[j2]]]);
#pragma unroll
      for (int u = 0; u < UP; u++)
        pv[u] = load_item<T, MODE>(J2.f, gmem(J2.X), J2.a.g.st[0], J2.a.g.st[1], bk2, bx2, its2,
                                   threadIdx.x + u * NT, J2.a.vec != 0, fast2,
                                   gmem(J2.code) + brick_start(J2.a.g, bk2), ppos[u]);
      Box lb2;
      lattice_box(bx2, lb2);
      if (threadIdx.x < (uint32_t)(lb2.E0 * lb2.b0))
        pcv = gmem(J2.cval)[(bn - begin[j2]) * kCoarseCells + threadIdx.x];
    }
    // compress: the lane's first lattice code, stored after the levels
    uint32_t pcc = 0;
    if (MODE == 0 && threadIdx.x < nlat) pcc = gmem(J.ccode)[bi * kCoarseCells + threadIdx.x];

    // ---- the levels below B with the block's configuration
    const hpez_interp c = a.cand[gmem(J.bcfg)[bi]];
    uint32_t nR = 0;
    if constexpr (PREF && FULL) {
      if (fast) {
        FBlock<T> fb{L,         code + brick_base, out,       lh,  hist, bk.o0, bk.o1, bk.o2, st0, st1,
                     bx.E0 - 1, bx.E1 - 1,         bx.E2 - 1, a.R, lo,   0.0,   0.0,   0.0,   0u};
        for (int l = a.L < kCoarseL ? a.L : kCoarseL; l >= 1; l--) {
          fb.el = a.el_l[l];
          fb.inv2e = a.inv2e_l[l];
          fb.twoe = a.twoe_l[l];
          if (l == 2) flevel<T, MODE, NT, 2>(c, fb, a.wmd);
          else flevel<T, MODE, NT, 1>(c, fb, a.wmd);
        }
        nR = fb.nR;
      }
    }
    if (!fast)
    for (int l = a.L < kCoarseL ? a.L : kCoarseL; l >= 1; l--) {
      const int32_t s = 1 << (l - 1);
      if (MODE == 0) {
        CompressOp<T> op{L,  code + brick_base, lh, hist, Eb1, Eb2, a.R, lo, a.el_l[l], a.inv2e_l[l],
                         a.twoe_l[l], 0u};
        box_level<T, NT>(c, bx, L, bk.o0, bk.o1, bk.o2, s, a.wmd, op);
        nR += op.nR;
      } else {
        DecompressOp<T> op{L, code + brick_base, out, bk.o0, bk.o1, bk.o2, st0, st1, Eb1, Eb2, a.R,
                           a.twoe_l[l]};
        box_level<T, NT>(c, bx, L, bk.o0, bk.o1, bk.o2, s, a.wmd, op);
      }
    }

    if (MODE == 1) {
      // the whole brick (interiors from the schedule, faces as loaded)
      const uint32_t nq2 = (uint32_t)((Eb2 + 3) >> 2);
      const uint32_t nitem = (uint32_t)(bk.Eb0 * Eb1) * nq2;
      const Divisor mg = fmagic(nq2);
      const Divisor mg1 = fmagic((uint32_t)Eb1);
      for (uint32_t it = threadIdx.x; it < nitem; it += NT) {
        const uint32_t r = fdiv(it, mg);
        const uint32_t q = it - r * nq2;
        const uint32_t c0 = fdiv(r, mg1);
        const uint32_t c1 = r - c0 * (uint32_t)Eb1;
        const int32_t cb = 4 * (int32_t)q;
        const int32_t cnt = Eb2 - cb < 4 ? Eb2 - cb : 4;
        HPEZ_GLOBAL T* dst = out + (bk.o0 + c0) * st0 + (bk.o1 + c1) * st1 + (bk.o2 + cb);
        const int32_t lb = fast ? fslot((int32_t)c0) * kFP0 + fslot((int32_t)c1) * kFP1 + (cb >> 1)
                                : (int32_t)(c0 * E1 + c1) * E2 + cb;
        if (fast) {
          // a full brick row: four cells at the even and odd slots of cb
          const T v0 = L[lb], v1 = L[lb + 17], v2 = L[lb + 1], v3 = L[lb + 18];
          if constexpr (sizeof(T) == 4) {
            if (vec) {
              *reinterpret_cast<HPEZ_GLOBAL vf4*>(dst) = vf4{v0, v1, v2, v3};
              continue;
            }
          }
          dst[0] = v0;
          dst[1] = v1;
          dst[2] = v2;
          dst[3] = v3;
        } else if (vec && cnt == 4) {
          if constexpr (sizeof(T) == 4) {
            const vf4 v = {(float)L[lb], (float)L[lb + 1], (float)L[lb + 2], (float)L[lb + 3]};
            *reinterpret_cast<HPEZ_GLOBAL vf4*>(dst) = v;
          } else {
            const vd2 v0 = {(double)L[lb], (double)L[lb + 1]};
            const vd2 v1 = {(double)L[lb + 2], (double)L[lb + 3]};
            reinterpret_cast<HPEZ_GLOBAL vd2*>(dst)[0] = v0;
            reinterpret_cast<HPEZ_GLOBAL vd2*>(dst)[1] = v1;
          }
        } else {
          for (int j = 0; j < cnt; j++) dst[j] = L[lb + j];
        }
      }
    } else {
      // the face codes into the brick, counted with the others
#pragma unroll
      for (int u = 0; u < FC; u++) {
        if (!fok[u]) continue;
        code[brick_base + fcd[u]] = (uint16_t)fcv[u];
        const uint32_t q = fcv[u];
        nR += q == a.R;
        if (q != a.R) {
          const uint32_t w = q - lo;
          if (w < (uint32_t)kBlockHistWin)
            __hip_atomic_fetch_add(&lh[w], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          else
            __hip_atomic_fetch_add(&hist[q], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      // the lattice points' codes (coarse levels) into the brick, counted too
      const HPEZ_GLOBAL uint16_t* cc = gmem(J.ccode) + bi * kCoarseCells;
      for (uint32_t i = threadIdx.x; i < nlat; i += NT) {
        const uint32_t q0 = fdiv(i, mlb0);
        const uint32_t r = i - q0 * (uint32_t)lb.b0;
        const uint32_t q1 = fdiv(r, mlE2);
        const int32_t i0 = (int32_t)q0, i1 = (int32_t)q1, i2 = (int32_t)(r - q1 * (uint32_t)lb.E2);
        if (i0 < lb.lo0 || i0 > lb.hi0 || i1 < lb.lo1 || i1 > lb.hi1 || i2 < lb.lo2 || i2 > lb.hi2)
          continue;
        const uint32_t q = i == threadIdx.x ? pcc : cc[i];
        code[brick_base + (uint32_t)((i0 * lk0 * Eb1 + i1 * lk1) * Eb2 + i2 * lk2)] = (uint16_t)q;
        nR += q == a.R;
        if (q != a.R) {
          const uint32_t w = q - lo;
          if (w < (uint32_t)kBlockHistWin)
            __hip_atomic_fetch_add(&lh[w], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          else
            __hip_atomic_fetch_add(&hist[q], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      // codes equal to R: a wave sum, then one LDS atomic per wave
      for (int o = 32; o > 0; o >>= 1) nR += __shfl_xor(nR, o, 64);
      if ((threadIdx.x & 63) == 0 && nR) {
        const uint32_t w = a.R - lo;
        if (w < (uint32_t)kBlockHistWin) atomicAdd(&lh[w], nR);
        else __hip_atomic_fetch_add(&hist[a.R], nR, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    gbi = bn;
  }
  if (MODE == 0 && hjob >= 0) {
    __syncthreads();
    hist_flush(lh, jobs[hjob], NT);
  }
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
hipError_t launch_face_steps(const FaceEntry<T>* d_tab, const uint64_t* d_wg_begin, int n,
                             uint64_t total_wg, bool narrow, int mode, uint32_t threads,
                             hipStream_t st)
{
  if (!total_wg || n <= 0) return hipSuccess;
  if (threads < 64 || threads > 256 || (threads & 63)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)total_wg), block(threads);
  if (mode == 0 && narrow)
    hipLaunchKernelGGL((face_step_kernel<T, 0, uint32_t>), grid, block, 0, st, d_tab, d_wg_begin, n);
  else if (mode == 0)
    hipLaunchKernelGGL((face_step_kernel<T, 0, uint64_t>), grid, block, 0, st, d_tab, d_wg_begin, n);
  else if (narrow)
    hipLaunchKernelGGL((face_step_kernel<T, 1, uint32_t>), grid, block, 0, st, d_tab, d_wg_begin, n);
  else
    hipLaunchKernelGGL((face_step_kernel<T, 1, uint64_t>), grid, block, 0, st, d_tab, d_wg_begin, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse_jobs(const BlockJobDev<T>* d_jobs, const uint64_t* d_begin, int n,
                              uint64_t total_blocks, int mode, hipStream_t st)
{
  if (!total_blocks || n <= 0) return hipSuccess;
  if (mode == 0)
    hipLaunchKernelGGL((coarse_kernel<T, 0>), dim3((unsigned)total_blocks), dim3(64), 0, st, d_jobs,
                       d_begin, n);
  else
    hipLaunchKernelGGL((coarse_kernel<T, 1>), dim3((unsigned)total_blocks), dim3(64), 0, st, d_jobs,
                       d_begin, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_planes(const PlaneJob<T>* d_tab, const uint64_t* d_wg_begin, int n,
                         uint64_t total_wg, size_t lds, int mode, hipStream_t st)
{
  if (!total_wg || n <= 0) return hipSuccess;
  if (mode == 0) {
    (void)hipFuncSetAttribute((const void*)plane_kernel<T, 0>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((plane_kernel<T, 0>), dim3((unsigned)total_wg), dim3(kBlockThreads), lds, st,
                       d_tab, d_wg_begin, n);
  } else {
    (void)hipFuncSetAttribute((const void*)plane_kernel<T, 1>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((plane_kernel<T, 1>), dim3((unsigned)total_wg), dim3(kBlockThreads), lds, st,
                       d_tab, d_wg_begin, n);
  }
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
  // float fields with full blocks hold them in the 33^3 slot layout
  if (sizeof(T) == 4 && g.act[0] && g.act[1] && g.act[2] && g.n[0] >= kBrick &&
      g.n[1] >= kBrick && g.n[2] >= kBrick)
    pts = (size_t)33 * kFP0;
  return ((pts * sizeof(T) + 15) & ~(size_t)15) + (size_t)kBlockHistWin * 4;
}

template <typename T, int NT>
void launch_block_kernel(const BlockJobDev<T>* d_jobs, const uint64_t* d_begin, int n, unsigned grid,
                         size_t lds, uint32_t lh_off, int mode, hipStream_t st)
{
  if (mode == 0) {
    (void)hipFuncSetAttribute((const void*)block_kernel<T, 0, NT>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((block_kernel<T, 0, NT>), dim3(grid), dim3(NT), lds, st, d_jobs, d_begin, n,
                       lh_off);
  } else {
    (void)hipFuncSetAttribute((const void*)block_kernel<T, 1, NT>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((block_kernel<T, 1, NT>), dim3(grid), dim3(NT), lds, st, d_jobs, d_begin, n,
                       lh_off);
  }
}

template <typename T>
hipError_t launch_block_jobs(const BlockJobDev<T>* d_jobs, const uint64_t* d_begin, int n,
                             uint64_t total_blocks, size_t lds, int n_cu, int mode, bool small,
                             hipStream_t st)
{
  if (!total_blocks || n <= 0) return hipSuccess;
  // persistent work-groups, blocks dealt round-robin (no work-group waits for
  // another): one per CU for any box (the box takes the CU's LDS), six per CU
  // for boxes of at most two active dims (measured: 4, 6, 8 per CU give 0.34,
  // 0.30, 0.31 ms on a 4096^2 float field); the histogram window takes the
  // last kBlockHistWin words
  if (lds < (size_t)kBlockHistWin * 4) return hipErrorInvalidValue;
  const uint32_t lh_off = (uint32_t)(lds - (size_t)kBlockHistWin * 4);
  const uint64_t per = small ? 6 * (uint64_t)n_cu : (uint64_t)n_cu;
  const unsigned grid = (unsigned)(total_blocks < per ? total_blocks : per);
  if (small)
    launch_block_kernel<T, kSmallBoxThreads>(d_jobs, d_begin, n, grid, lds, lh_off, mode, st);
  else
    launch_block_kernel<T, kBlockThreads>(d_jobs, d_begin, n, grid, lds, lh_off, mode, st);
  return hipGetLastError();
}

#define INST(T)                                                                                  \
  template hipError_t launch_face_init<T>(const FaceGeo&, const Geom&, const Lattice&, const T*, \
                                          const uint16_t*, int, hipStream_t);                    \
  template size_t block_lds_bytes<T>(const Geom&);                                               \
  template hipError_t launch_planes<T>(const PlaneJob<T>*, const uint64_t*, int, uint64_t, size_t,  \
                                       int, hipStream_t);                                         \
  template hipError_t launch_coarse_jobs<T>(const BlockJobDev<T>*, const uint64_t*, int, uint64_t, \
                                            int, hipStream_t);                                     \
  template hipError_t launch_block_jobs<T>(const BlockJobDev<T>*, const uint64_t*, int, uint64_t, \
                                           size_t, int, int, bool, hipStream_t);                  \
  template hipError_t launch_face_steps<T>(const FaceEntry<T>*, const uint64_t*, int, uint64_t,   \
                                           bool, int, uint32_t, hipStream_t);                     \
  template hipError_t launch_minmax_faces<T>(const T*, const Geom&, const FaceGeo&, double*, int*, \
                                             int, hipStream_t);
INST(float)
INST(double)

}  // namespace hpez
