// k_codec.hip -- single-pass Huffman encode and table-driven decode (gfx950).
//
// Encode: one wavefront per chunk of `chunk` symbols, chunks taken in order
// from a ticket counter.  Each lane sums the code lengths of its run of
// symbols; a wave prefix sum gives the chunk's bit count, and the chunk's bit
// offset comes from a decoupled look-back over the chunks before it (each
// chunk publishes its count, then its inclusive prefix; a chunk only waits on
// chunks with smaller tickets, which are already running, so every wait ends).
// The codewords are assembled in LDS and written out as whole 32-bit words;
// only the two words a chunk shares with its neighbours are OR-ed atomically
// into the zeroed payload.
//
// Decode: one lane per chunk; a 2^12-entry first-level table in LDS resolves
// codewords up to 12 bits in one lookup; codes are packed eight at a time into
// 16-byte stores.

#include "codec_dev.h"
#include "interp_dev.h"

namespace hpez {

constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagIncl = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;
constexpr int kEncWaves = 4;  // chunks per work-group

__device__ __forceinline__ uint64_t ld_acquire(const uint64_t* p)
{
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(uint64_t* p, uint64_t v)
{
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(256) encode1_kernel(EncodeArgs a, const uint16_t* __restrict__ code,
                                                      uint32_t* __restrict__ words,
                                                      uint16_t* __restrict__ out_cb,
                                                      uint64_t* __restrict__ flags,
                                                      uint32_t* __restrict__ ticket,
                                                      const uint32_t* __restrict__ gtab)
{
  // codebook window in LDS: entry = codeword << 6 | length (lengths <= 32, codewords < 2^26
  // when the table is used; longer codes fall back to the global table)
  __shared__ uint32_t tab[kEncTab];
  __shared__ uint32_t buf[kEncWaves][kEncWords];
  __shared__ uint32_t tk[kEncWaves];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (a.lds_tab)
    for (uint32_t i = threadIdx.x; i < a.ntab; i += blockDim.x) tab[i] = gtab[i];
  if (lane == 0) tk[w] = atomicAdd(ticket, 1u);
  __syncthreads();
  const uint64_t k = tk[w];
  if (k >= a.nch) return;
  const uint32_t per = a.chunk / 64;
  const uint64_t beg = k * a.chunk + (uint64_t)lane * per;
  const uint64_t cend = k * a.chunk + a.chunk < a.n ? k * a.chunk + a.chunk : a.n;
  uint32_t ent[16];
  uint32_t bits = 0;
  for (uint32_t j = 0; j < per; j++) {
    const uint64_t i = beg + j;
    uint32_t e = 0;
    if (i < cend) {
      const uint32_t c = code[i] - a.smin;
      e = a.lds_tab ? tab[c] : gtab[c];
    }
    ent[j] = e;
    bits += e & 63u;
  }
  // wave prefix sum of the lanes' bit counts
  uint32_t incl = bits;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  const uint32_t total = __shfl(incl, 63, 64);
  const uint32_t lane_off = incl - bits;
  // look-back for the chunk's bit offset
  uint64_t excl = 0;
  if (lane == 0) {
    if (k == 0) {
      st_release(&flags[0], kFlagIncl | total);
    } else {
      st_release(&flags[k], kFlagAgg | total);
      int64_t j = (int64_t)k - 1;
      for (;;) {
        uint64_t f;
        do {
          f = ld_acquire(&flags[j]);
        } while (f == 0);
        excl += f & kValMask;
        if ((f & ~kValMask) == kFlagIncl) break;
        j--;
      }
      st_release(&flags[k], kFlagIncl | (excl + total));
    }
    out_cb[k] = (uint16_t)total;
  }
  excl = __shfl(excl, 0, 64);
  // assemble in LDS: local bit 0 is global bit (excl & ~31)
  const uint32_t sh = (uint32_t)(excl & 31);
  const uint32_t nw = (sh + total + 31) / 32;
  uint32_t* B = buf[w];
  for (uint32_t i = lane; i < nw + 1; i += 64) B[i] = 0;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  uint32_t pos = sh + lane_off;
  for (uint32_t j = 0; j < per; j++) {
    const uint32_t e = ent[j];
    const uint32_t L = e & 63u;
    if (L) {
      const uint32_t cw = e >> 6;
      const uint32_t wi = pos >> 5, off = pos & 31;
      const uint64_t v = (uint64_t)cw << (64 - L - off);
      const uint32_t hi = (uint32_t)(v >> 32), lo = (uint32_t)v;
      if (hi) atomicOr(&B[wi], hi);
      if (lo) atomicOr(&B[wi + 1], lo);
      pos += L;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const uint64_t w0 = excl >> 5;
  for (uint32_t i = lane; i < nw; i += 64) {
    const uint32_t v = B[i];
    if (i == 0 || i == nw - 1) {
      if (v) atomicOr(&words[w0 + i], v);
    } else {
      words[w0 + i] = v;
    }
  }
}

// long codewords (> 26 bits) cannot use the packed table: a plain global one
__global__ void __launch_bounds__(256) encode1_wide_kernel(EncodeArgs a, const uint16_t* __restrict__ code,
                                                           uint32_t* __restrict__ words,
                                                           uint16_t* __restrict__ out_cb,
                                                           uint64_t* __restrict__ flags,
                                                           uint32_t* __restrict__ ticket,
                                                           const uint8_t* __restrict__ len,
                                                           const uint32_t* __restrict__ cw)
{
  __shared__ uint32_t tk[kEncWaves];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) tk[w] = atomicAdd(ticket, 1u);
  __syncthreads();
  const uint64_t k = tk[w];
  if (k >= a.nch) return;
  const uint32_t per = a.chunk / 64;
  const uint64_t beg = k * a.chunk + (uint64_t)lane * per;
  const uint64_t cend = k * a.chunk + a.chunk < a.n ? k * a.chunk + a.chunk : a.n;
  uint32_t bits = 0;
  for (uint32_t j = 0; j < per; j++)
    if (beg + j < cend) bits += len[code[beg + j]];
  uint32_t incl = bits;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  const uint32_t total = __shfl(incl, 63, 64);
  uint64_t excl = 0;
  if (lane == 0) {
    if (k == 0) {
      st_release(&flags[0], kFlagIncl | total);
    } else {
      st_release(&flags[k], kFlagAgg | total);
      int64_t j = (int64_t)k - 1;
      for (;;) {
        uint64_t f;
        do {
          f = ld_acquire(&flags[j]);
        } while (f == 0);
        excl += f & kValMask;
        if ((f & ~kValMask) == kFlagIncl) break;
        j--;
      }
      st_release(&flags[k], kFlagIncl | (excl + total));
    }
    out_cb[k] = (uint16_t)total;
  }
  excl = __shfl(excl, 0, 64);
  uint64_t pos = excl + (incl - bits);
  for (uint32_t j = 0; j < per; j++) {
    if (beg + j >= cend) break;
    const uint32_t c = code[beg + j];
    const uint32_t L = len[c];
    const uint64_t wi = pos >> 5;
    const uint32_t off = (uint32_t)(pos & 31);
    const uint64_t v = (uint64_t)cw[c] << (64 - L - off);
    const uint32_t hi = (uint32_t)(v >> 32), lo = (uint32_t)v;
    if (hi) atomicOr(&words[wi], hi);
    if (lo) atomicOr(&words[wi + 1], lo);
    pos += L;
  }
}

hipError_t launch_encode1(const EncodeArgs& a, const uint16_t* code, uint32_t* words,
                          uint16_t* out_cb, uint64_t* flags, uint32_t* ticket,
                          const uint32_t* packed, const uint8_t* len, const uint32_t* cw,
                          hipStream_t st)
{
  if (!a.nch) return hipSuccess;
  const unsigned grid = (unsigned)((a.nch + kEncWaves - 1) / kEncWaves);
  if (a.packed_ok)
    hipLaunchKernelGGL(encode1_kernel, dim3(grid), dim3(64 * kEncWaves), 0, st, a, code, words,
                       out_cb, flags, ticket, packed);
  else
    hipLaunchKernelGGL(encode1_wide_kernel, dim3(grid), dim3(64 * kEncWaves), 0, st, a, code, words,
                       out_cb, flags, ticket, len, cw);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// verbatim values (code 0) in stream order: chunks with zeros walk their codes
template <typename T>
__global__ void __launch_bounds__(256) gather_unpred_kernel(const uint16_t* __restrict__ code, uint64_t n,
                                                            uint32_t chunk, const uint32_t* __restrict__ czero,
                                                            const uint64_t* __restrict__ zoff,
                                                            const T* __restrict__ X, T* __restrict__ unpred,
                                                            Geom g, uint64_t nch)
{
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nch || czero[k] == 0) return;
  const uint64_t beg = k * chunk;
  const uint64_t end = beg + chunk < n ? beg + chunk : n;
  uint64_t z = zoff[k];
  for (uint64_t i = beg; i < end; i++) {
    if (code[i] != 0) continue;
    int64_t x[4];
    brick_coords(g.n, (int64_t)i, x);
    unpred[z++] = X[x[0] * g.st[0] + x[1] * g.st[1] + x[2] * g.st[2] + x[3]];
  }
}

__global__ void __launch_bounds__(256) count_zero_kernel(const uint16_t* __restrict__ code, uint64_t n,
                                                         uint32_t chunk, uint32_t* __restrict__ czero,
                                                         uint64_t nch)
{
  const uint64_t k = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= nch) return;
  const int lane = threadIdx.x & 63;
  const uint64_t beg = k * chunk;
  const uint64_t end = beg + chunk < n ? beg + chunk : n;
  uint32_t z = 0;
  for (uint64_t i = beg + lane; i < end; i += 64) z += code[i] == 0;
  for (int o = 32; o > 0; o >>= 1) z += __shfl_xor(z, o, 64);
  if (lane == 0) czero[k] = z;
}

template <typename T>
hipError_t launch_gather_unpred(const uint16_t* code, uint64_t n, uint32_t chunk, uint32_t* czero,
                                uint64_t* zoff, uint64_t* tmp, const T* X, T* unpred, const Geom& g,
                                hipStream_t st)
{
  const uint64_t nch = (n + chunk - 1) / chunk;
  if (!nch) return hipSuccess;
  hipLaunchKernelGGL(count_zero_kernel, dim3((unsigned)((nch + 3) / 4)), dim3(256), 0, st, code, n, chunk,
                     czero, nch);
  hipError_t e = launch_scan_u32_to_u64(czero, nch, zoff, zoff + nch, tmp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((gather_unpred_kernel<T>), dim3((unsigned)((nch + 255) / 256)), dim3(256), 0, st,
                     code, n, chunk, czero, zoff, X, unpred, g, nch);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// decode
__global__ void __launch_bounds__(256) decode2_kernel(DecodeArgs a, const uint32_t* __restrict__ words,
                                                      const uint64_t* __restrict__ bit_off,
                                                      const uint32_t* __restrict__ glut,
                                                      const uint32_t* __restrict__ first,
                                                      const uint32_t* __restrict__ count,
                                                      const uint32_t* __restrict__ offset,
                                                      const uint16_t* __restrict__ sorted,
                                                      uint16_t* __restrict__ code,
                                                      uint32_t* __restrict__ czero,
                                                      int* __restrict__ status)
{
  __shared__ uint32_t lut[1 << kLutBits];
  __shared__ uint32_t s_first[kLmax + 2], s_count[kLmax + 2], s_offset[kLmax + 2];
  for (int i = threadIdx.x; i < (1 << kLutBits); i += blockDim.x) lut[i] = glut[i];
  for (int i = threadIdx.x; i < kLmax + 2; i += blockDim.x) {
    s_first[i] = first[i];
    s_count[i] = count[i];
    s_offset[i] = offset[i];
  }
  __syncthreads();
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0 && bit_off[a.nch] != a.nbits) atomicOr(status, 1);
  if (k >= a.nch) return;
  const uint64_t beg = k * a.chunk;
  const uint64_t end = beg + a.chunk < a.n ? beg + a.chunk : a.n;
  uint64_t pos = bit_off[k];
  const uint64_t stop = k + 1 < a.nch ? bit_off[k + 1] : bit_off[a.nch];
  if (stop > a.nbits) {
    atomicOr(status, 1);
    return;
  }
  const uint64_t nwords = (a.nbits + 31) / 32;
  uint64_t wi = pos >> 5;
  uint64_t buf;
  int have;
  {
    const uint32_t skip = (uint32_t)(pos & 31);
    const uint64_t w = wi < nwords ? words[wi] : 0;
    buf = (w << 32) << skip;
    have = 32 - (int)skip;
    wi++;
  }
  uint32_t zeros = 0;
  bool bad = false;
  uint32_t pack[4] = {0, 0, 0, 0};
  const bool aligned = (beg & 7) == 0;
  for (uint64_t i = beg; i < end; i++) {
    if (have < 32) {
      const uint64_t w = wi < nwords ? words[wi] : 0;
      buf |= (w << 32) >> have;
      have += 32;
      wi++;
    }
    const uint32_t e = lut[(uint32_t)(buf >> (64 - kLutBits))];
    uint32_t sym, L = e & 0xFFu;
    if (L) {
      sym = e >> 8;
    } else {
      sym = 0;
      for (uint32_t l = kLutBits + 1; l <= (uint32_t)kLmax; l++) {
        const uint32_t v = (uint32_t)(buf >> (64 - l));
        if (s_count[l] && v - s_first[l] < s_count[l]) {
          L = l;
          sym = sorted[s_offset[l] + (v - s_first[l])];
          break;
        }
      }
      if (!L) {
        bad = true;
        break;
      }
    }
    zeros += sym == 0;
    buf <<= L;
    have -= (int)L;
    pos += L;
    const uint32_t slot = (uint32_t)(i - beg) & 7u;
    if (aligned) {
      pack[slot >> 1] |= sym << ((slot & 1) * 16);
      if (slot == 7 || i + 1 == end) {
        const uint64_t base = i & ~7ull;
        if (slot == 7) {
          *reinterpret_cast<uint4*>(code + base) = make_uint4(pack[0], pack[1], pack[2], pack[3]);
        } else {
          for (uint32_t t = 0; t <= slot; t++) code[base + t] = (uint16_t)(pack[t >> 1] >> ((t & 1) * 16));
        }
        pack[0] = pack[1] = pack[2] = pack[3] = 0;
      }
    } else {
      code[i] = (uint16_t)sym;
    }
  }
  if (bad || pos != stop) atomicOr(status, 1);
  czero[k] = zeros;
}

hipError_t launch_decode2(const DecodeArgs& a, const uint32_t* words, const uint64_t* bit_off,
                          const uint32_t* lut, const uint32_t* first, const uint32_t* count,
                          const uint32_t* offset, const uint16_t* sorted, uint16_t* code,
                          uint32_t* czero, int* status, hipStream_t st)
{
  if (!a.nch) return hipSuccess;
  hipLaunchKernelGGL(decode2_kernel, dim3((unsigned)((a.nch + 255) / 256)), dim3(256), 0, st, a, words,
                     bit_off, lut, first, count, offset, sorted, code, czero, status);
  return hipGetLastError();
}

template hipError_t launch_gather_unpred<float>(const uint16_t*, uint64_t, uint32_t, uint32_t*,
                                                uint64_t*, uint64_t*, const float*, float*,
                                                const Geom&, hipStream_t);
template hipError_t launch_gather_unpred<double>(const uint16_t*, uint64_t, uint32_t, uint32_t*,
                                                 uint64_t*, uint64_t*, const double*, double*,
                                                 const Geom&, hipStream_t);

}  // namespace hpez
