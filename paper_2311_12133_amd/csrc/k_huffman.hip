// k_huffman.hip -- histogram, Huffman encode and chunk-parallel decode of the
// quantization codes (Sec. 4, step 4), gfx950.
//
// Stream conventions (shared with the host runtime): canonical codewords,
// most significant bit first, bit p of the payload is bit 31 - p%32 of 32-bit
// word p/32, symbols in row-major order, no padding between chunks of `chunk`
// symbols; the stream stores each chunk's bit count so chunks decode in
// parallel.

#include "interp_dev.h"

namespace hpez {

// ---------------------------------------------------------------------------
// histogram: a window of bins around the zero-error symbol R lives in LDS
// (quantization codes concentrate there); everything else goes straight to
// global atomics.
constexpr int kHistWin = 4096;

__global__ void __launch_bounds__(256) histogram_kernel(const uint16_t* __restrict__ code,
                                                        uint64_t n, uint32_t* __restrict__ hist,
                                                        uint32_t lo)
{
  __shared__ uint32_t h[kHistWin];
  for (int i = threadIdx.x; i < kHistWin; i += 256) h[i] = 0;
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint32_t c = code[i];
    const uint32_t w = c - lo;
    if (w < (uint32_t)kHistWin) atomicAdd(&h[w], 1u);
    else atomicAdd(&hist[c], 1u);
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
  hipLaunchKernelGGL(histogram_kernel, dim3((unsigned)blocks), dim3(256), 0, st, code, n, hist, lo);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// wave-level helpers (wavefront of 64 lanes)
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t* total)
{
  const int lane = threadIdx.x & 63;
  uint32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  *total = __shfl(x, 63, 64);
  return x - v;
}

// per-chunk bit counts and counts of code 0 (verbatim values)
__global__ void __launch_bounds__(256) chunk_lengths_kernel(const uint16_t* __restrict__ code,
                                                            uint64_t n, uint32_t chunk,
                                                            const uint8_t* __restrict__ len,
                                                            uint32_t* __restrict__ cbits,
                                                            uint32_t* __restrict__ czero,
                                                            uint64_t nch)
{
  const uint64_t k = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= nch) return;
  const int lane = threadIdx.x & 63;
  const uint64_t beg = k * chunk;
  const uint64_t end = beg + chunk < n ? beg + chunk : n;
  uint32_t bits = 0, zeros = 0;
  for (uint64_t i = beg + lane; i < end; i += 64) {
    const uint32_t c = code[i];
    bits += len[c];
    zeros += c == 0;
  }
  for (int o = 32; o > 0; o >>= 1) {
    bits += __shfl_xor(bits, o, 64);
    zeros += __shfl_xor(zeros, o, 64);
  }
  if (lane == 0) {
    cbits[k] = bits;
    czero[k] = zeros;
  }
}

hipError_t launch_chunk_lengths(const uint16_t* code, uint64_t n, uint32_t chunk,
                                const uint8_t* d_len, uint32_t* chunk_bits, uint32_t* chunk_zero,
                                hipStream_t st)
{
  const uint64_t nch = (n + chunk - 1) / chunk;
  if (nch == 0) return hipSuccess;
  hipLaunchKernelGGL(chunk_lengths_kernel, dim3((unsigned)((nch + 3) / 4)), dim3(256), 0, st, code,
                     n, chunk, d_len, chunk_bits, chunk_zero, nch);
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

__global__ void __launch_bounds__(256) zero_words_kernel(uint32_t* __restrict__ w,
                                                         const uint64_t* __restrict__ total_bits)
{
  const uint64_t nw = (*total_bits + 31) / 32;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += stride) w[i] = 0;
}

hipError_t launch_zero_words(uint32_t* words, const uint64_t* d_total_bits, hipStream_t st)
{
  hipLaunchKernelGGL(zero_words_kernel, dim3(1024), dim3(256), 0, st, words, d_total_bits);
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

// ---------------------------------------------------------------------------
// encode: one wavefront per chunk; each lane owns a run of consecutive
// symbols, a wave prefix sum gives every lane its first bit, codewords are
// OR-ed into the zeroed payload.  Code-0 points copy their original value to
// the verbatim section in row-major order.
__device__ __forceinline__ void put_code(uint32_t* __restrict__ words, uint64_t pos, uint32_t cw,
                                         uint32_t L)
{
  const uint64_t w = pos >> 5;
  const uint32_t off = (uint32_t)(pos & 31);
  // codeword occupies bits [off, off + L) of the 64-bit window starting at word w
  const uint64_t v = (uint64_t)cw << (64 - L - off);
  const uint32_t hi = (uint32_t)(v >> 32), lo = (uint32_t)v;
  if (hi) atomicOr(&words[w], hi);
  if (lo) atomicOr(&words[w + 1], lo);
}

template <typename T>
__global__ void __launch_bounds__(256) encode_kernel(
    const uint16_t* __restrict__ code, uint64_t n, uint32_t chunk, const uint8_t* __restrict__ len,
    const uint32_t* __restrict__ cw, const uint64_t* __restrict__ bit_off,
    const uint64_t* __restrict__ zero_off, const uint32_t* __restrict__ cbits,
    const uint32_t* __restrict__ czero, uint32_t* __restrict__ words, uint16_t* __restrict__ out_cb,
    const T* __restrict__ X, T* __restrict__ unpred, uint64_t nch, Geom g)
{
  const uint64_t k = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= nch) return;
  const int lane = threadIdx.x & 63;
  const uint32_t per = chunk / 64;
  const uint64_t beg = k * chunk + (uint64_t)lane * per;
  const uint64_t cend = k * chunk + chunk < n ? k * chunk + chunk : n;
  const uint64_t end = beg + per < cend ? beg + per : cend;
  uint32_t bits = 0, zeros = 0;
  for (uint64_t i = beg; i < end; i++) {
    const uint32_t c = code[i];
    bits += len[c];
    zeros += c == 0;
  }
  uint32_t tb, tz;
  const uint32_t pb = wave_excl_scan(bits, &tb);
  const uint32_t pz = wave_excl_scan(zeros, &tz);
  uint64_t pos = bit_off[k] + pb;
  uint64_t zp = zero_off[k] + pz;
  for (uint64_t i = beg; i < end; i++) {
    const uint32_t c = code[i];
    const uint32_t L = len[c];
    put_code(words, pos, cw[c], L);
    pos += L;
    if (c == 0 && unpred) {
      int64_t x[4];
      brick_coords(g.n, (int64_t)i, x);
      unpred[zp++] = X[x[0] * g.st[0] + x[1] * g.st[1] + x[2] * g.st[2] + x[3]];
    }
  }
  if (lane == 0) out_cb[k] = (uint16_t)cbits[k];
  (void)czero;
}

template <typename T>
hipError_t launch_encode(const uint16_t* code, uint64_t n, uint32_t chunk, const uint8_t* d_len,
                         const uint32_t* d_cw, const uint64_t* bit_off, const uint64_t* zero_off,
                         const uint32_t* chunk_bits, const uint32_t* chunk_zero, uint32_t* payload,
                         uint16_t* out_chunk_bits, const T* X, T* out_unpred, const Geom& g,
                         hipStream_t st)
{
  const uint64_t nch = (n + chunk - 1) / chunk;
  if (nch == 0) return hipSuccess;
  hipLaunchKernelGGL((encode_kernel<T>), dim3((unsigned)((nch + 3) / 4)), dim3(256), 0, st, code, n,
                     chunk, d_len, d_cw, bit_off, zero_off, chunk_bits, chunk_zero, payload,
                     out_chunk_bits, X, out_unpred, nch, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// decode: one lane per chunk.  A 12-bit first-level table resolves short
// codewords in one lookup; longer ones walk the canonical (first code, count)
// table per length.  Lanes check that each chunk consumes exactly its stored
// bit count.
template <typename T>
__global__ void __launch_bounds__(256) decode_kernel(
    const uint32_t* __restrict__ words, uint64_t nbits, const uint64_t* __restrict__ bit_off,
    uint64_t n, uint32_t chunk, const uint32_t* __restrict__ lut, const uint32_t* __restrict__ first,
    const uint32_t* __restrict__ count, const uint32_t* __restrict__ offset,
    const uint16_t* __restrict__ sorted, uint16_t* __restrict__ code, uint32_t* __restrict__ czero,
    int* __restrict__ status, uint64_t nch, const uint64_t* __restrict__ total_bits)
{
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0 && *total_bits != nbits) atomicOr(status, 1);
  if (k >= nch) return;
  const uint64_t beg = k * chunk;
  const uint64_t end = beg + chunk < n ? beg + chunk : n;
  uint64_t pos = bit_off[k];
  const uint64_t stop = k + 1 < nch ? bit_off[k + 1] : *total_bits;
  if (stop > nbits) {
    atomicOr(status, 1);
    return;
  }
  const uint64_t nwords = (nbits + 31) / 32;
  // bit buffer: `buf` holds the next `have` bits, left-aligned
  uint64_t buf = 0;
  int have = 0;
  uint64_t wi = pos >> 5;
  {
    const uint32_t skip = (uint32_t)(pos & 31);
    const uint64_t w = wi < nwords ? words[wi] : 0;
    buf = (w << 32) << skip;
    have = 32 - (int)skip;
    wi++;
  }
  uint32_t zeros = 0;
  bool bad = false;
  for (uint64_t i = beg; i < end; i++) {
    if (have < 32) {
      const uint64_t w = wi < nwords ? words[wi] : 0;
      buf |= (w << 32) >> have;
      have += 32;
      wi++;
    }
    const uint32_t peek = (uint32_t)(buf >> (64 - kLutBits));
    const uint32_t e = lut[peek];
    uint32_t sym, L;
    if (e & 0xFFu) {
      L = e & 0xFFu;
      sym = e >> 8;
    } else {
      L = 0;
      sym = 0;
      for (uint32_t l = kLutBits + 1; l <= (uint32_t)kLmax; l++) {
        const uint32_t v = (uint32_t)(buf >> (64 - l));
        if (count[l] && v - first[l] < count[l]) {
          L = l;
          sym = sorted[offset[l] + (v - first[l])];
          break;
        }
      }
      if (!L) {
        bad = true;
        break;
      }
    }
    code[i] = (uint16_t)sym;
    zeros += sym == 0;
    buf <<= L;
    have -= (int)L;
    pos += L;
  }
  if (bad || pos != stop) atomicOr(status, 1);
  czero[k] = zeros;
}

template <typename T>
hipError_t launch_decode(const uint32_t* payload, uint64_t nbits, const uint64_t* bit_off,
                         uint64_t n, uint32_t chunk, const uint32_t* d_lut, const uint32_t* d_first,
                         const uint32_t* d_count, const uint32_t* d_offset, const uint16_t* d_sorted,
                         uint16_t* code, uint32_t* chunk_zero, int* d_status, hipStream_t st)
{
  const uint64_t nch = (n + chunk - 1) / chunk;
  if (nch == 0) return hipSuccess;
  // the scan's total sits right after the offsets (see the host runtime)
  hipLaunchKernelGGL((decode_kernel<T>), dim3((unsigned)((nch + 255) / 256)), dim3(256), 0, st,
                     payload, nbits, bit_off, n, chunk, d_lut, d_first, d_count, d_offset, d_sorted,
                     code, chunk_zero, d_status, nch, bit_off + nch);
  return hipGetLastError();
}

// verbatim values back into place: lanes of chunks that hold code-0 points walk
// their chunk in row-major order, skipping anchors.
template <typename T>
__global__ void __launch_bounds__(256) scatter_unpred_kernel(
    const uint16_t* __restrict__ code, uint64_t n, uint32_t chunk, const uint32_t* __restrict__ czero,
    const uint64_t* __restrict__ zero_off, const T* __restrict__ unpred, uint64_t n_unpred,
    T* __restrict__ W, int* __restrict__ status, uint64_t nch, Geom g)
{
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nch || czero[k] == 0) return;
  const uint64_t beg = k * chunk;
  const uint64_t end = beg + chunk < n ? beg + chunk : n;
  uint64_t z = zero_off[k];
  for (uint64_t i = beg; i < end; i++) {
    if (code[i] != 0) continue;
    if (z >= n_unpred) {
      atomicOr(status, 1);
      return;
    }
    int64_t x[4];
    brick_coords(g.n, (int64_t)i, x);
    W[x[0] * g.st[0] + x[1] * g.st[1] + x[2] * g.st[2] + x[3]] = unpred[z++];
  }
}

template <typename T>
hipError_t launch_scatter_unpred(const uint16_t* code, uint64_t n, uint32_t chunk,
                                 const uint32_t* chunk_zero, const uint64_t* zero_off,
                                 const T* unpred, uint64_t n_unpred, T* W, int* d_status,
                                 const Geom& g, hipStream_t st)
{
  const uint64_t nch = (n + chunk - 1) / chunk;
  if (nch == 0) return hipSuccess;
  hipLaunchKernelGGL((scatter_unpred_kernel<T>), dim3((unsigned)((nch + 255) / 256)), dim3(256), 0,
                     st, code, n, chunk, chunk_zero, zero_off, unpred, n_unpred, W, d_status, nch, g);
  return hipGetLastError();
}

#define INST(T)                                                                                    \
  template hipError_t launch_encode<T>(const uint16_t*, uint64_t, uint32_t, const uint8_t*,        \
                                       const uint32_t*, const uint64_t*, const uint64_t*,          \
                                       const uint32_t*, const uint32_t*, uint32_t*, uint16_t*,     \
                                       const T*, T*, const Geom&, hipStream_t);                    \
  template hipError_t launch_decode<T>(const uint32_t*, uint64_t, const uint64_t*, uint64_t,       \
                                       uint32_t, const uint32_t*, const uint32_t*,                 \
                                       const uint32_t*, const uint32_t*, const uint16_t*,          \
                                       uint16_t*, uint32_t*, int*, hipStream_t);                   \
  template hipError_t launch_scatter_unpred<T>(const uint16_t*, uint64_t, uint32_t,                \
                                               const uint32_t*, const uint64_t*, const T*,         \
                                               uint64_t, T*, int*, const Geom&, hipStream_t);
INST(float)
INST(double)

}  // namespace hpez
