// k_lossless.hip -- the byte passes of the lossless stage after Huffman
// coding (Sec. 4, step 5): nonzero-byte compaction, zero-run tokens with
// their histogram, and the expansion of decoded tokens.  Every pass is a
// plain data-parallel map or compaction; the entropy coding of the tokens is
// the quantization codes' Huffman encoder and decoder.
#include "lossless_dev.h"

namespace hpez {

namespace {

constexpr int kLT = 256;                        // threads per work-group
constexpr int kLPer = (int)(kLLTile / kLT);     // bytes per thread (16)

// the kLPer bytes of thread t of tile `tile` (zero past n); one 16-byte load
// when the whole run is in range and aligned
__device__ __forceinline__ void load16(const uint8_t* __restrict__ b, uint64_t n, uint64_t i,
                                       uint8_t* v)
{
  if (i + kLPer <= n && ((reinterpret_cast<uintptr_t>(b + i) & 15) == 0)) {
    const uint4 w = *reinterpret_cast<const uint4*>(b + i);
    const uint32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int k = 0; k < kLPer; k++) v[k] = (uint8_t)(u[k >> 2] >> (8 * (k & 3)));
  } else {
#pragma unroll
    for (int k = 0; k < kLPer; k++) v[k] = i + k < n ? b[i + k] : 0;
  }
}

// exclusive prefix of v over the work-group (in thread order) and the total
__device__ __forceinline__ uint32_t wg_excl(uint32_t v, uint32_t* total)
{
  __shared__ uint32_t wsum[kLT / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t incl = v;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int w = 0; w < kLT / 64; w++) {
    if (w < wv) before += wsum[w];
    all += wsum[w];
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

__global__ void __launch_bounds__(kLT) ll_count_kernel(const uint8_t* __restrict__ b, uint64_t n,
                                                       uint32_t* __restrict__ cnt)
{
  uint8_t v[kLPer];
  load16(b, n, (uint64_t)blockIdx.x * kLLTile + threadIdx.x * kLPer, v);
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < kLPer; k++) c += v[k] != 0;
  uint32_t tot;
  (void)wg_excl(c, &tot);
  if (threadIdx.x == 0) cnt[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kLT) ll_compact_kernel(const uint8_t* __restrict__ b, uint64_t n,
                                                         const uint64_t* __restrict__ tile_off,
                                                         uint32_t* __restrict__ pos)
{
  const uint64_t i0 = (uint64_t)blockIdx.x * kLLTile + threadIdx.x * kLPer;
  uint8_t v[kLPer];
  load16(b, n, i0, v);
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < kLPer; k++) c += v[k] != 0;
  uint32_t tot;
  uint64_t o = tile_off[blockIdx.x] + wg_excl(c, &tot);
#pragma unroll
  for (int k = 0; k < kLPer; k++)
    if (v[k]) pos[o++] = (uint32_t)(i0 + k);
}

__global__ void __launch_bounds__(kLT) ll_tokcount_kernel(const uint32_t* __restrict__ pos,
                                                          const uint64_t* __restrict__ nnz_p,
                                                          uint64_t n, uint32_t* __restrict__ tcnt)
{
  const uint64_t j = (uint64_t)blockIdx.x * kLT + threadIdx.x;
  if (j > n) return;
  const uint64_t nnz = *nnz_p;
  if (j > nnz) {
    tcnt[j] = 0;
    return;
  }
  const int64_t prev = j ? (int64_t)pos[j - 1] : -1;
  const int64_t next = j < nnz ? (int64_t)pos[j] : (int64_t)n;
  const uint64_t gap = (uint64_t)(next - prev - 1);
  tcnt[j] = (uint32_t)(gap / kRunMax + (gap % kRunMax ? 1 : 0) + (j < nnz ? 1 : 0));
}

__global__ void __launch_bounds__(kLT) ll_tokens_kernel(const uint8_t* __restrict__ b,
                                                        const uint32_t* __restrict__ pos,
                                                        const uint64_t* __restrict__ nnz_p,
                                                        uint64_t n, const uint64_t* __restrict__ toff,
                                                        uint16_t* __restrict__ tok,
                                                        uint32_t* __restrict__ hist)
{
  __shared__ uint32_t lh[kTokSyms];
  for (uint32_t i = threadIdx.x; i < kTokSyms; i += kLT) lh[i] = 0;
  __syncthreads();
  const uint64_t nnz = *nnz_p;
  // grid-stride over the nonzero bytes (and the run after the last one), so
  // that few work-groups clear and flush the LDS histogram
  for (uint64_t j = (uint64_t)blockIdx.x * kLT + threadIdx.x; j <= nnz && j <= n;
       j += (uint64_t)gridDim.x * kLT) {
    const int64_t prev = j ? (int64_t)pos[j - 1] : -1;
    const int64_t next = j < nnz ? (int64_t)pos[j] : (int64_t)n;
    const uint64_t gap = (uint64_t)(next - prev - 1);
    uint64_t o = toff[j];
    const uint64_t full = gap / kRunMax;
    const uint32_t r = (uint32_t)(gap % kRunMax);
    for (uint64_t k = 0; k < full; k++) tok[o++] = (uint16_t)(255 + kRunMax);
    if (full) atomicAdd(&lh[255 + kRunMax], (uint32_t)full);
    if (r) {
      tok[o++] = (uint16_t)(255 + r);
      atomicAdd(&lh[255 + r], 1u);
    }
    if (j < nnz) {
      const uint32_t v = b[next];
      tok[o] = (uint16_t)v;
      atomicAdd(&lh[v], 1u);
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < kTokSyms; i += kLT)
    if (lh[i]) atomicAdd(&hist[i], lh[i]);
}

__global__ void __launch_bounds__(kLT) ll_toklen_kernel(const uint16_t* __restrict__ tok, uint64_t ntok,
                                                        uint32_t* __restrict__ len,
                                                        int* __restrict__ status)
{
  const uint64_t t = (uint64_t)blockIdx.x * kLT + threadIdx.x;
  if (t >= ntok) return;
  const uint32_t v = tok[t];
  const bool ok = v >= 1 && v <= 255 + kRunMax;
  if (!ok) atomicOr(status, 1);
  len[t] = !ok ? 0u : v <= 255 ? 1u : v - 255;
}

__global__ void __launch_bounds__(kLT) ll_expand_kernel(const uint16_t* __restrict__ tok, uint64_t ntok,
                                                        const uint64_t* __restrict__ off,
                                                        uint8_t* __restrict__ out, uint64_t n,
                                                        int* __restrict__ status)
{
  const uint64_t t = (uint64_t)blockIdx.x * kLT + threadIdx.x;
  if (t >= ntok) return;
  const uint32_t v = tok[t];
  if (v < 1 || v > 255) return;  // runs: the output is zeroed
  const uint64_t o = off[t];
  if (o < n) out[o] = (uint8_t)v;
  else atomicOr(status, 1);
}

unsigned grid_of(uint64_t threads) { return (unsigned)((threads + kLT - 1) / kLT); }

}  // namespace

hipError_t launch_ll_count(const uint8_t* b, uint64_t n, uint32_t* cnt, hipStream_t st)
{
  const uint64_t nt = (n + kLLTile - 1) / kLLTile;
  if (nt) hipLaunchKernelGGL(ll_count_kernel, dim3((unsigned)nt), dim3(kLT), 0, st, b, n, cnt);
  return hipGetLastError();
}

hipError_t launch_ll_compact(const uint8_t* b, uint64_t n, const uint64_t* tile_off, uint32_t* pos,
                             hipStream_t st)
{
  const uint64_t nt = (n + kLLTile - 1) / kLLTile;
  if (nt)
    hipLaunchKernelGGL(ll_compact_kernel, dim3((unsigned)nt), dim3(kLT), 0, st, b, n, tile_off, pos);
  return hipGetLastError();
}

hipError_t launch_ll_tokcount(const uint32_t* pos, const uint64_t* nnz, uint64_t n, uint32_t* tcnt,
                              hipStream_t st)
{
  hipLaunchKernelGGL(ll_tokcount_kernel, dim3(grid_of(n + 1)), dim3(kLT), 0, st, pos, nnz, n, tcnt);
  return hipGetLastError();
}

hipError_t launch_ll_tokens(const uint8_t* b, const uint32_t* pos, const uint64_t* nnz, uint64_t n,
                            const uint64_t* toff, uint16_t* tok, uint32_t* hist, hipStream_t st)
{
  const unsigned g = grid_of(n + 1) < 2048u ? grid_of(n + 1) : 2048u;
  hipLaunchKernelGGL(ll_tokens_kernel, dim3(g), dim3(kLT), 0, st, b, pos, nnz, n, toff, tok, hist);
  return hipGetLastError();
}

hipError_t launch_ll_toklen(const uint16_t* tok, uint64_t ntok, uint32_t* len, int* status,
                            hipStream_t st)
{
  if (ntok)
    hipLaunchKernelGGL(ll_toklen_kernel, dim3(grid_of(ntok)), dim3(kLT), 0, st, tok, ntok, len,
                       status);
  return hipGetLastError();
}

hipError_t launch_ll_expand(const uint16_t* tok, uint64_t ntok, const uint64_t* off, uint8_t* out,
                            uint64_t n, int* status, hipStream_t st)
{
  if (ntok)
    hipLaunchKernelGGL(ll_expand_kernel, dim3(grid_of(ntok)), dim3(kLT), 0, st, tok, ntok, off, out,
                       n, status);
  return hipGetLastError();
}

}  // namespace hpez
