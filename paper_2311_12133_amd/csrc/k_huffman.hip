// k_huffman.hip -- code histogram (Sec. 4, step 4) and the exclusive scans
// the coder uses (chunk bit offsets, counts of verbatim values), gfx950.

#include "interp_dev.h"

namespace hpez {

// ---------------------------------------------------------------------------
// histogram: a window of bins around the zero-error symbol R lives in LDS
// (quantization codes concentrate there); everything else goes straight to
// global atomics.
constexpr int kHistWin = 4096;

// Codes R - 1, R and R + 1 (most of them on smooth data, so lanes of a
// wavefront would contend for the same LDS bin) are counted in registers and
// added once per lane at the end; the rest go to the LDS window or global.
// Lanes read eight codes at a time when the array is 16-byte aligned.
__global__ void __launch_bounds__(256) histogram_kernel(const uint16_t* __restrict__ code,
                                                        uint64_t n, uint32_t* __restrict__ hist,
                                                        uint32_t lo, uint32_t R)
{
  __shared__ uint32_t h[kHistWin];
  for (int i = threadIdx.x; i < kHistWin; i += 256) h[i] = 0;
  __syncthreads();
  uint32_t near[3] = {0, 0, 0};
  auto add = [&](uint32_t c) {
    const uint32_t d = c - (R - 1);
    if (d < 3) {
      near[0] += d == 0;
      near[1] += d == 1;
      near[2] += d == 2;
    } else {
      const uint32_t w = c - lo;
      if (w < (uint32_t)kHistWin) atomicAdd(&h[w], 1u);
      else atomicAdd(&hist[c], 1u);
    }
  };
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t done = 0;
  if ((reinterpret_cast<uintptr_t>(code) & 15) == 0) {
    const uint64_t ng = n / 8;
    const uint4* v8 = reinterpret_cast<const uint4*>(code);
    for (uint64_t g = gid; g < ng; g += stride) {
      const uint4 v = v8[g];
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int k = 0; k < 4; k++) {
        add(w[k] & 0xffffu);
        add(w[k] >> 16);
      }
    }
    done = ng * 8;
  }
  for (uint64_t i = done + gid; i < n; i += stride) add(code[i]);
#pragma unroll
  for (int k = 0; k < 3; k++) {
    uint32_t c = near[k];
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0 && c) {
      const uint32_t b = R - 1 + (uint32_t)k, w = b - lo;
      if (w < (uint32_t)kHistWin) atomicAdd(&h[w], c);
      else atomicAdd(&hist[b], c);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kHistWin; i += 256)
    if (h[i]) atomicAdd(&hist[lo + i], h[i]);
}

hipError_t launch_histogram(const uint16_t* code, uint64_t n, uint32_t* hist, uint32_t nsym,
                            uint32_t R, hipStream_t st)
{
  uint32_t lo = R > kHistWin / 2 ? R - kHistWin / 2 : 0;
  if (lo + kHistWin > nsym) lo = nsym > (uint32_t)kHistWin ? nsym - kHistWin : 0;
  uint64_t blocks = (n + 256 * 16 - 1) / (256 * 16);
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(histogram_kernel, dim3((unsigned)blocks), dim3(256), 0, st, code, n, hist, lo,
                     R);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// exclusive scan u32 -> u64 (three phases: tile sums, scan of tile sums, tiles)
constexpr int kScanTile = 1024;

__global__ void __launch_bounds__(256) scan_tile_sums(const uint32_t* __restrict__ in, uint64_t n,
                                                      uint64_t* __restrict__ sums)
{
  __shared__ uint64_t s[256];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  uint64_t acc = 0;
  for (int j = 0; j < 4; j++) {
    const uint64_t i = base + threadIdx.x * 4 + j;
    if (i < n) acc += in[i];
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(256) scan_sums_kernel(uint64_t* __restrict__ sums, uint64_t nt,
                                                        uint64_t* __restrict__ total)
{
  __shared__ uint64_t s[256];
  __shared__ uint64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint64_t base = 0; base < nt; base += 256) {
    const uint64_t i = base + threadIdx.x;
    const uint64_t v = i < nt ? sums[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      const uint64_t y = (int)threadIdx.x >= o ? s[threadIdx.x - o] : 0;
      __syncthreads();
      s[threadIdx.x] += y;
      __syncthreads();
    }
    if (i < nt) sums[i] = carry + s[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += s[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(256) scan_tiles_kernel(const uint32_t* __restrict__ in, uint64_t n,
                                                         const uint64_t* __restrict__ sums,
                                                         uint64_t* __restrict__ out)
{
  __shared__ uint64_t s[256];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  uint64_t v[4], acc = 0;
  for (int j = 0; j < 4; j++) {
    const uint64_t i = base + threadIdx.x * 4 + j;
    v[j] = i < n ? in[i] : 0;
    acc += v[j];
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const uint64_t y = (int)threadIdx.x >= o ? s[threadIdx.x - o] : 0;
    __syncthreads();
    s[threadIdx.x] += y;
    __syncthreads();
  }
  uint64_t run = sums[blockIdx.x] + s[threadIdx.x] - acc;
  for (int j = 0; j < 4; j++) {
    const uint64_t i = base + threadIdx.x * 4 + j;
    if (i < n) out[i] = run;
    run += v[j];
  }
}

hipError_t launch_scan_u32_to_u64(const uint32_t* in, uint64_t n, uint64_t* out_excl,
                                  uint64_t* d_total, uint64_t* tmp, hipStream_t st)
{
  const uint64_t nt = (n + kScanTile - 1) / kScanTile;
  if (nt == 0) return hipMemsetAsync(d_total, 0, 8, st);
  hipLaunchKernelGGL(scan_tile_sums, dim3((unsigned)nt), dim3(256), 0, st, in, n, tmp);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(256), 0, st, tmp, nt, d_total);
  hipLaunchKernelGGL(scan_tiles_kernel, dim3((unsigned)nt), dim3(256), 0, st, in, n, tmp, out_excl);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) u16_to_u32_kernel(const uint16_t* __restrict__ in, uint64_t n,
                                                         uint32_t* __restrict__ out)
{
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = in[i];
}

hipError_t launch_u16_to_u32(const uint16_t* in, uint64_t n, uint32_t* out, hipStream_t st)
{
  if (!n) return hipSuccess;
  uint64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(u16_to_u32_kernel, dim3((unsigned)b), dim3(256), 0, st, in, n, out);
  return hipGetLastError();
}

}  // namespace hpez
