// k_codec.hip -- single-pass Huffman encode and table-driven decode (gfx950).
//
// Encode: one wavefront per chunk of `chunk` symbols, chunks taken in order
// from a ticket counter by persistent waves.  Each lane sums the code lengths
// of its run of symbols; a wave prefix sum gives the chunk's bit count, and the
// chunk's bit offset comes from a decoupled look-back over the chunks before it
// (each chunk publishes its count, then its inclusive prefix; a chunk only
// waits on chunks with smaller tickets, whose waves took them earlier and are
// running, and a wave publishes its count before it waits, so every wait ends).
// The codewords are assembled in LDS and written out as whole 32-bit words;
// only the two words a chunk shares with its neighbours are OR-ed atomically
// into the zeroed payload.
//
// Decode: one lane per chunk; a 2^12-entry first-level table in LDS resolves
// codewords up to 12 bits in one lookup, longer ones are found by comparing the
// window with the per-length limits of the canonical code (uniform values, no
// table walk); codes are packed eight at a time into 16-byte stores.

#include <algorithm>

#include "codec_dev.h"
#include "interp_dev.h"

namespace hpez {

constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagIncl = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;
constexpr int kEncWaves = 4;  // chunks per work-group

// A flag word carries its own payload (status bits + bit count), and no other
// data is published through it, so relaxed device-scope atomics suffice: they
// are coherent across the chip's L2 slices without cache maintenance, which
// acquire/release ordering would add to every poll.
__device__ __forceinline__ uint64_t flag_load(const uint64_t* p)
{
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void flag_store(uint64_t* p, uint64_t v)
{
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive bit offset of chunk k by decoupled look-back, run by the whole
// wave: each round reads the flags of the 64 chunks before the current window
// end, waits until all of them are published, and stops at the nearest one that
// carries an inclusive prefix.  Called after chunk k published its aggregate.
__device__ __forceinline__ uint64_t look_back(uint64_t* flags, uint64_t k, int lane)
{
  uint64_t excl = 0;
  int64_t top = (int64_t)k - 1;
  for (;;) {
    const int64_t j = top - lane;
    uint64_t f = j >= 0 ? flag_load(&flags[j]) : kFlagIncl;
    while (__ballot(f == 0)) {
      __builtin_amdgcn_s_sleep(1);
      if (f == 0) f = flag_load(&flags[j]);
    }
    const uint64_t incl = __ballot((f & ~kValMask) == kFlagIncl);
    // lanes up to (and including) the nearest inclusive flag contribute
    const int stop = incl ? __builtin_ctzll(incl) : 64;
    uint64_t v = lane <= stop ? (f & kValMask) : 0;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    excl += v;
    if (incl) return excl;
    top -= 64;
  }
}

// the length of a packed entry (escaped long codewords from the long table)
__device__ __forceinline__ uint32_t ent_len(uint32_t e, const uint64_t* __restrict__ ltab)
{
  const uint32_t L = e & 63u;
  return L == 63u ? (uint32_t)(ltab[e >> 6] & 63u) : L;
}

// bit count of one chunk (lane sums of `per` symbols, wave total); ent[]
// receives the packed entries of the lane's symbols
// the PER codes of one lane of a full chunk of 64 PER symbols (PER 8 or 16;
// 16-byte aligned runs)
template <int PER>
struct RawN {
  uint4 v[PER / 8];
};
template <int PER>
__device__ __forceinline__ RawN<PER> raw_load(const uint16_t* __restrict__ code, uint64_t k, int lane)
{
  const uint4* p = reinterpret_cast<const uint4*>(code + k * (64 * PER) + (uint64_t)lane * PER);
  RawN<PER> r;
#pragma unroll
  for (int q = 0; q < PER / 8; q++) r.v[q] = p[q];
  return r;
}
template <int PER>
__device__ __forceinline__ uint32_t raw_entries(const EncodeArgs& a, const uint32_t* tab,
                                                const uint32_t* __restrict__ gtab,
                                                const RawN<PER>& r, uint32_t* ent,
                                                uint32_t& lane_bits)
{
  uint32_t w[PER / 2];
#pragma unroll
  for (int q = 0; q < PER / 8; q++) {
    w[4 * q] = r.v[q].x;
    w[4 * q + 1] = r.v[q].y;
    w[4 * q + 2] = r.v[q].z;
    w[4 * q + 3] = r.v[q].w;
  }
  uint32_t bits = 0;
#pragma unroll
  for (int j = 0; j < PER; j++) {
    const uint32_t c = ((w[j >> 1] >> ((j & 1) * 16)) & 0xFFFFu) - a.smin;
    const uint32_t e = a.lds_tab ? tab[c] : gtab[c];
    ent[j] = e;
    bits += ent_len(e, a.ltab);
  }
  lane_bits = bits;
  uint32_t t = bits;
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
  return t;
}

__device__ __forceinline__ uint32_t chunk_entries(const EncodeArgs& a, const uint16_t* __restrict__ code,
                                                  const uint32_t* tab, const uint32_t* __restrict__ gtab,
                                                  uint64_t k, int lane, uint32_t* ent, uint32_t& lane_bits)
{
  const uint32_t per = a.chunk / 64;
  const uint64_t beg = k * a.chunk + (uint64_t)lane * per;
  const uint64_t cend = k * a.chunk + a.chunk < a.n ? k * a.chunk + a.chunk : a.n;
  uint32_t bits = 0;
  if (per == 16 && k * a.chunk + a.chunk <= a.n) {
    // the lane's 16 codes in two 16-byte loads (32-byte aligned run)
    const uint4* p = reinterpret_cast<const uint4*>(code + beg);
    const uint4 v0 = p[0], v1 = p[1];
    const uint32_t w[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
    for (int j = 0; j < 16; j++) {
      const uint32_t c = ((w[j >> 1] >> ((j & 1) * 16)) & 0xFFFFu) - a.smin;
      const uint32_t e = a.lds_tab ? tab[c] : gtab[c];
      ent[j] = e;
      bits += ent_len(e, a.ltab);
    }
  } else {
    for (uint32_t j = 0; j < per; j++) {
      const uint64_t i = beg + j;
      uint32_t e = 0;
      if (i < cend) {
        const uint32_t c = code[i] - a.smin;
        e = a.lds_tab ? tab[c] : gtab[c];
      }
      ent[j] = e;
      bits += ent_len(e, a.ltab);
    }
  }
  lane_bits = bits;
  uint32_t t = bits;
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
  return t;
}

// Packs one chunk whose first bit is global bit `excl`: the wave assembles the
// chunk in its LDS buffer B (local bit 0 is global bit excl & ~31) and writes it
// as whole 32-bit words; the two words the chunk may share with its neighbours
// are OR-ed atomically into the zeroed payload.  A lane whose run fits in 128
// bits builds it in registers and ORs at most four words into B; a longer run
// falls back to one or two LDS ORs per codeword.
__device__ __forceinline__ void pack_chunk(uint32_t* B, uint32_t* __restrict__ words, uint64_t excl,
                                           uint32_t total, uint32_t lb, const uint32_t* ent,
                                           uint32_t per, int lane, const uint64_t* __restrict__ ltab)
{
  uint32_t incl = lb;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  const uint32_t lane_off = incl - lb;
  const uint32_t sh = (uint32_t)(excl & 31);
  const uint32_t nw = (sh + total + 31) / 32;
  __builtin_amdgcn_wave_barrier();
  for (uint32_t i = lane; i < nw + 1; i += 64) B[i] = 0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  uint32_t pos = sh + lane_off;
  const uint32_t off0 = pos & 31;
  if (off0 + lb <= 128) {
    unsigned __int128 acc = 0;
    for (uint32_t jj = 0; jj < per; jj++) {
      const uint32_t e = ent[jj];
      uint64_t le = e;
      if ((e & 63u) == 63u) le = ltab[e >> 6];
      acc = (acc << (le & 63u)) | (unsigned __int128)(le >> 6);
    }
    if (lb) {
      acc <<= 128 - off0 - lb;
      const uint32_t wi = pos >> 5;
      const uint32_t nwl = (off0 + lb + 31) >> 5;
#pragma unroll
      for (uint32_t q = 0; q < 4; q++) {
        const uint32_t v = (uint32_t)(acc >> (96 - 32 * q));
        if (q < nwl && v) atomicOr(&B[wi + q], v);
      }
    }
  } else {
    for (uint32_t jj = 0; jj < per; jj++) {
      const uint32_t e = ent[jj];
      uint64_t le = e;
      if ((e & 63u) == 63u) le = ltab[e >> 6];
      const uint32_t L = (uint32_t)(le & 63u);
      if (L) {
        const uint64_t cw = le >> 6;
        const uint32_t wi = pos >> 5, off = pos & 31;
        const uint64_t v = cw << (64 - L - off);
        const uint32_t hi = (uint32_t)(v >> 32), lo = (uint32_t)v;
        if (hi) atomicOr(&B[wi], hi);
        if (lo) atomicOr(&B[wi + 1], lo);
        pos += L;
      }
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

// Persistent work-groups take partitions of kPart chunks in ticket order.  A
// partition's chunk bit counts are summed in LDS, one decoupled look-back per
// partition gives its bit offset, then each wave packs its chunks.  Full
// partitions keep each wave's kEncCpw chunks of codes in registers from the
// counting pass to the packing pass, so the codes are read from memory once;
// the ragged last partition reads them again.  The codebook window lives in
// LDS once per work-group.
constexpr int kEncCpw = 8;                   // chunks per wave and partition
constexpr int kPart = kEncWaves * kEncCpw;   // chunks per partition

template <int PER>
__global__ void __launch_bounds__(256) encode1_kernel(EncodeArgs a, const uint16_t* __restrict__ code,
                                                      uint32_t* __restrict__ words,
                                                      uint16_t* __restrict__ out_cb,
                                                      uint64_t* __restrict__ flags,
                                                      uint32_t* __restrict__ ticket,
                                                      const uint32_t* __restrict__ gtab)
{
  // codebook window in LDS: entry = codeword << 6 | length (codewords < 2^26)
  __shared__ uint32_t tab[kEncTab];
  __shared__ uint32_t buf[kEncWaves][kEncWords];
  __shared__ uint32_t cbits[kPart];
  __shared__ uint64_t s_excl;
  __shared__ uint32_t s_part;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (a.lds_tab)
    for (uint32_t i = threadIdx.x; i < a.ntab; i += blockDim.x) tab[i] = gtab[i];
  const uint64_t nparts = (a.nch + kPart - 1) / kPart;
  uint32_t* B = buf[w];
  const uint32_t per = a.chunk / 64;
  for (;;) {
    if (threadIdx.x == 0) s_part = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint64_t part = s_part;
    if (part >= nparts) return;
    const uint64_t k0 = part * kPart;
    const uint32_t np = (uint32_t)(a.nch - k0 < (uint64_t)kPart ? a.nch - k0 : (uint64_t)kPart);
    uint32_t ent[16];
    // full chunks of 64 PER symbols, all of them complete
    const bool fast = a.chunk == 64 * PER && np == (uint32_t)kPart && (k0 + np) * (64 * PER) <= a.n;
    RawN<PER> raw[kEncCpw];
    // 1. chunk bit counts
    if (fast) {
#pragma unroll
      for (int c = 0; c < kEncCpw; c++) raw[c] = raw_load<PER>(code, k0 + w + c * kEncWaves, lane);
#pragma unroll
      for (int c = 0; c < kEncCpw; c++) {
        const uint32_t j = w + c * kEncWaves;
        uint32_t lb;
        const uint32_t t = raw_entries<PER>(a, tab, gtab, raw[c], ent, lb);
        if (lane == 0) {
          cbits[j] = t;
          out_cb[k0 + j] = (uint16_t)t;
        }
      }
    } else {
      for (uint32_t j = w; j < np; j += kEncWaves) {
        uint32_t lb;
        const uint32_t t = chunk_entries(a, code, tab, gtab, k0 + j, lane, ent, lb);
        if (lane == 0) {
          cbits[j] = t;
          out_cb[k0 + j] = (uint16_t)t;
        }
      }
    }
    __syncthreads();
    // 2. partition prefix and look-back (wave 0)
    if (w == 0) {
      const uint32_t v = (uint32_t)lane < np ? cbits[lane] : 0u;
      uint32_t incl = v;
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
      }
      const uint64_t total = __shfl(incl, 63, 64);
      if ((uint32_t)lane < np) cbits[lane] = incl - v;  // exclusive prefix inside the partition
      uint64_t excl = 0;
      if (part == 0) {
        if (lane == 0) flag_store(&flags[0], kFlagIncl | total);
      } else {
        if (lane == 0) flag_store(&flags[part], kFlagAgg | total);
        excl = look_back(flags, part, lane);
        if (lane == 0) flag_store(&flags[part], kFlagIncl | (excl + total));
      }
      if (lane == 0) s_excl = excl;
    }
    __syncthreads();
    // 3. pack each chunk
    const uint64_t pexcl = s_excl;
    if (fast) {
#pragma unroll
      for (int c = 0; c < kEncCpw; c++) {
        const uint32_t j = w + c * kEncWaves;
        uint32_t lb;
        const uint32_t total = raw_entries<PER>(a, tab, gtab, raw[c], ent, lb);
        pack_chunk(B, words, pexcl + cbits[j], total, lb, ent, PER, lane, a.ltab);
      }
    } else {
      for (uint32_t j = w; j < np; j += kEncWaves) {
        uint32_t lb;
        const uint32_t total = chunk_entries(a, code, tab, gtab, k0 + j, lane, ent, lb);
        pack_chunk(B, words, pexcl + cbits[j], total, lb, ent, per, lane, a.ltab);
      }
    }
    __syncthreads();
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
  const int lane = threadIdx.x & 63;
  const uint32_t per = a.chunk / 64;
  for (;;) {
    uint32_t t = 0;
    if (lane == 0) t = atomicAdd(ticket, 1u);
    const uint64_t k = (uint64_t)__shfl(t, 0, 64);
    if (k >= a.nch) return;
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
    if (k == 0) {
      if (lane == 0) flag_store(&flags[0], kFlagIncl | total);
    } else {
      if (lane == 0) flag_store(&flags[k], kFlagAgg | total);
      excl = look_back(flags, k, lane);
      if (lane == 0) flag_store(&flags[k], kFlagIncl | (excl + total));
    }
    if (lane == 0) out_cb[k] = (uint16_t)total;
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
}

// ---------------------------------------------------------------------------
// copies and fills of the stream's small sections in one launch (grid y: the
// segment); 8-byte words, then the last n % 8 bytes one by one

__global__ void __launch_bounds__(256) byte_segs_kernel(ByteSegs a)
{
  const ByteSeg g = a.s[blockIdx.y];
  const uint64_t nw = g.n / 8;
  uint64_t* __restrict__ d = reinterpret_cast<uint64_t*>(g.dst);
  const uint64_t* __restrict__ sp = reinterpret_cast<const uint64_t*>(g.src);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += stride)
    d[i] = sp ? sp[i] : 0ull;
  if (blockIdx.x == 0 && threadIdx.x < (g.n & 7)) {
    const uint64_t k = nw * 8 + threadIdx.x;
    g.dst[k] = g.src ? g.src[k] : (uint8_t)0;
  }
}

hipError_t launch_byte_segs(const ByteSegs& a, hipStream_t st)
{
  if (a.count <= 0) return hipSuccess;
  uint64_t most = 0;
  for (int i = 0; i < a.count; i++) most = std::max<uint64_t>(most, a.s[i].n / 8);
  uint64_t gx = (most + 255) / 256;
  gx = gx < 1 ? 1 : (gx > 1024 ? 1024 : gx);
  hipLaunchKernelGGL(byte_segs_kernel, dim3((unsigned)gx, (unsigned)a.count), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_encode1(const EncodeArgs& a, const uint16_t* code, uint32_t* words,
                          uint16_t* out_cb, uint64_t* flags, uint32_t* ticket,
                          const uint32_t* packed, const uint8_t* len, const uint32_t* cw,
                          hipStream_t st)
{
  if (!a.nch) return hipSuccess;
  if (a.packed_ok) {
    // persistent grid: a few work-groups per CU, each taking partitions in order
    const uint64_t want = (a.nch + kPart - 1) / kPart;
    const unsigned grid = (unsigned)(want < 1024 ? want : 1024);
    if (a.chunk == 512)
      hipLaunchKernelGGL(encode1_kernel<8>, dim3(grid), dim3(64 * kEncWaves), 0, st, a, code, words,
                         out_cb, flags, ticket, packed);
    else
      hipLaunchKernelGGL(encode1_kernel<16>, dim3(grid), dim3(64 * kEncWaves), 0, st, a, code,
                         words, out_cb, flags, ticket, packed);
  } else {
    const uint64_t want = (a.nch + kEncWaves - 1) / kEncWaves;
    const unsigned grid = (unsigned)(want < 2048 ? want : 2048);
    hipLaunchKernelGGL(encode1_wide_kernel, dim3(grid), dim3(64 * kEncWaves), 0, st, a, code, words,
                       out_cb, flags, ticket, len, cw);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Verbatim values (code 0) in stream order.  One wavefront per chunk; chunks
// without zeros return at once.  The lanes read 64 consecutive codes per round
// and rank the zeros among them with a ballot, so the values move in order.
// GATHER: X -> unpred (compress); otherwise unpred -> W (decompress, with the
// rank checked against the stored count).
template <typename T, bool GATHER>
__global__ void __launch_bounds__(256) unpred_move_kernel(const uint16_t* __restrict__ code, uint64_t n,
                                                          uint32_t chunk, const uint32_t* __restrict__ czero,
                                                          const uint64_t* __restrict__ zoff,
                                                          const T* __restrict__ src, T* __restrict__ dst,
                                                          uint64_t n_unpred, int* __restrict__ status,
                                                          Geom g, uint64_t nch)
{
  const uint64_t k = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= nch || czero[k] == 0) return;
  const int lane = threadIdx.x & 63;
  const uint64_t beg = k * chunk;
  const uint64_t end = beg + chunk < n ? beg + chunk : n;
  uint64_t z = zoff[k];
  for (uint64_t i0 = beg; i0 < end; i0 += 64) {
    const uint64_t i = i0 + lane;
    const bool zero = i < end && code[i] == 0;
    const uint64_t m = __ballot(zero);
    if (zero) {
      const uint64_t r = z + (uint64_t)__popcll(m & ((1ull << lane) - 1));
      int64_t x[4];
      brick_coords(g.n, (int64_t)i, x);
      const int64_t idx = x[0] * g.st[0] + x[1] * g.st[1] + x[2] * g.st[2] + x[3];
      if (GATHER) {
        dst[r] = src[idx];
      } else if (r < n_unpred) {
        dst[idx] = src[r];
      } else {
        atomicOr(status, 1);
      }
    }
    z += (uint64_t)__popcll(m);
  }
}

// zeros per chunk: 16-byte loads of eight codes when the chunk allows
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
  if (end - beg == chunk && chunk >= 512) {
    // 8 codes per lane per round
    for (uint64_t i = beg + (uint64_t)lane * 8; i < end; i += 512) {
      const uint4 v = *reinterpret_cast<const uint4*>(code + i);
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < 4; j++) z += ((w[j] & 0xFFFFu) == 0) + ((w[j] >> 16) == 0);
    }
  } else {
    for (uint64_t i = beg + lane; i < end; i += 64) z += code[i] == 0;
  }
  for (int o = 32; o > 0; o >>= 1) z += __shfl_xor(z, o, 64);
  if (lane == 0) czero[k] = z;
}

hipError_t launch_count_zeros(const uint16_t* code, uint64_t n, uint32_t chunk, uint32_t* czero,
                              uint64_t* zoff, uint64_t* tmp, hipStream_t st)
{
  const uint64_t nch = (n + chunk - 1) / chunk;
  if (!nch) return hipSuccess;
  hipLaunchKernelGGL(count_zero_kernel, dim3((unsigned)((nch + 3) / 4)), dim3(256), 0, st, code, n, chunk,
                     czero, nch);
  return launch_scan_u32_to_u64(czero, nch, zoff, zoff + nch, tmp, st);
}

template <typename T>
hipError_t launch_gather_unpred(const uint16_t* code, uint64_t n, uint32_t chunk, uint32_t* czero,
                                uint64_t* zoff, uint64_t* tmp, const T* X, T* unpred, const Geom& g,
                                hipStream_t st)
{
  const uint64_t nch = (n + chunk - 1) / chunk;
  if (!nch) return hipSuccess;
  hipError_t e = launch_count_zeros(code, n, chunk, czero, zoff, tmp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((unpred_move_kernel<T, true>), dim3((unsigned)((nch + 3) / 4)), dim3(256), 0, st,
                     code, n, chunk, czero, zoff, X, unpred, (uint64_t)0, (int*)nullptr, g, nch);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scatter_unpred2(const uint16_t* code, uint64_t n, uint32_t chunk,
                                  const uint32_t* czero, const uint64_t* zoff, const T* unpred,
                                  uint64_t n_unpred, T* W, int* d_status, const Geom& g,
                                  hipStream_t st)
{
  const uint64_t nch = (n + chunk - 1) / chunk;
  if (!nch) return hipSuccess;
  hipLaunchKernelGGL((unpred_move_kernel<T, false>), dim3((unsigned)((nch + 3) / 4)), dim3(256), 0,
                     st, code, n, chunk, czero, zoff, unpred, W, n_unpred, d_status, g, nch);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// decode

// symbol of the codeword at the top of the window; L = its length (0: invalid).
// Codes longer than the table are located by the canonical limits and read
// from the LDS copy of their symbols (or the global one when too many).
// MODE 0: codes longer than the first-level table by the canonical limits,
// their symbols in LDS; 1: the same with the symbols in global memory; 2:
// second-level tables in LDS first (a prefix without a code has entry 0), the
// limits for codes longer than the second level (their symbols in LDS when
// they fit).
template <int MODE>
__device__ __forceinline__ uint32_t decode_one(const DecodeArgs& a, const uint32_t* lut,
                                               const uint16_t* slong,
                                               const uint16_t* __restrict__ sorted,
                                               const uint32_t* subl, const uint32_t* sbase,
                                               uint32_t w, uint32_t& L)
{
  const uint32_t e = lut[w >> (32 - kLutBits)];
  L = e & 0xFFu;
  if (MODE == 2) {
    if (!(L & 0x80u)) return e >> 8;
    const uint32_t k = L & 0x7Fu;
    const uint32_t e2 = subl[(e >> 8) + ((w << kLutBits) >> (32 - k))];
    L = e2 & 0xFFu;
    if (L) return e2 >> 8;
    // longer than the second level (or no code): by the limits below
  }
  if (L) return e >> 8;
  // longer than the table: count the limits at or below w (they are sorted)
  uint32_t c = kLutBits + 1;
#pragma unroll
  for (int l = kLutBits + 1; l <= kLmax; l++) c += (uint64_t)w >= a.lim[l] ? 1u : 0u;
  if (c > (uint32_t)kLmax) {
    L = 0;
    return 0;
  }
  L = c;
  const uint32_t idx = sbase[c] + (w >> (32 - c));
  if (MODE == 0 || (MODE == 2 && a.n_long <= kDecLong)) return slong[idx - a.long_first];
  return sorted[idx];
}

constexpr uint32_t kDecRing = 16;  // LDS ring slots per decoding lane (a power of two)

template <int MODE>
__global__ void __launch_bounds__(256) decode2_kernel(DecodeArgs a, const uint32_t* __restrict__ words,
                                                      const uint16_t* __restrict__ cbits,
                                                      uint64_t* __restrict__ tflags,
                                                      const uint32_t* __restrict__ glut,
                                                      const uint16_t* __restrict__ sorted,
                                                      const uint32_t* __restrict__ gsub,
                                                      uint16_t* __restrict__ code,
                                                      uint32_t* __restrict__ czero,
                                                      int* __restrict__ status)
{
  __shared__ uint32_t lut[1 << kLutBits];
  __shared__ uint16_t slong[MODE != 1 ? kDecLong : 1];
  __shared__ uint32_t subl[MODE == 2 ? kDecSub : 1];
  __shared__ uint32_t ring[kDecRing * 256];
  // per-length offsets, indexed by a computed length (an LDS read instead of
  // a load from the kernel arguments)
  __shared__ uint32_t sbase[kLmax + 1];
  if (threadIdx.x <= (unsigned)kLmax) sbase[threadIdx.x] = a.base[threadIdx.x];
  for (int i = threadIdx.x; i < (1 << kLutBits); i += blockDim.x) lut[i] = glut[i];
  if (MODE == 0 || (MODE == 2 && a.n_long <= kDecLong))
    for (uint32_t i = threadIdx.x; i < a.n_long; i += blockDim.x) slong[i] = sorted[a.long_first + i];
  if (MODE == 2)
    for (uint32_t i = threadIdx.x; i < a.n_sub; i += blockDim.x) subl[i] = gsub[i];
  // Chunk bit offsets: work-groups take tiles of 256 chunks in ticket order
  // (status[1] is the ticket), scan the tile's bit counts and find the tile's
  // offset by decoupled look-back over the tiles before it (tflags, zeroed).
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_wsum[4];
  __shared__ uint64_t s_excl;
  if (threadIdx.x == 0) s_tile = atomicAdd(reinterpret_cast<uint32_t*>(status) + 1, 1u);
  __syncthreads();
  const uint64_t tile = s_tile;
  const uint64_t k = tile * 256 + threadIdx.x;
  const uint32_t cnt = k < a.nch ? (uint32_t)cbits[k] : 0u;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t incl = cnt;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) s_wsum[wv] = incl;
  __syncthreads();
  uint32_t before = 0;
  for (int w = 0; w < wv; w++) before += s_wsum[w];
  if (wv == 0) {
    const uint64_t agg = (uint64_t)s_wsum[0] + s_wsum[1] + s_wsum[2] + s_wsum[3];
    uint64_t excl = 0;
    if (tile == 0) {
      if (lane == 0) flag_store(&tflags[0], kFlagIncl | agg);
    } else {
      if (lane == 0) flag_store(&tflags[tile], kFlagAgg | agg);
      excl = look_back(tflags, tile, lane);
      if (lane == 0) flag_store(&tflags[tile], kFlagIncl | (excl + agg));
    }
    if (lane == 0) s_excl = excl;
  }
  __syncthreads();
  if (k >= a.nch) return;
  const uint64_t beg = k * a.chunk;
  const uint64_t end = beg + a.chunk < a.n ? beg + a.chunk : a.n;
  uint64_t pos = s_excl + before + (incl - cnt);
  const uint64_t stop = pos + cnt;
  if (k == a.nch - 1 && stop != a.nbits) atomicOr(status, 1);
  if (stop > a.nbits || pos > stop) {
    atomicOr(status, 1);
    return;
  }
  const uint64_t nwords = (a.nbits + 31) / 32;
  if (nwords == 0) {
    if (end > beg) atomicOr(status, 1);
    czero[k] = 0;
    return;
  }
  // 64-bit bit buffer, next bit at the top; `have` valid bits; `pre` holds the
  // payload word rd, the next one to enter the buffer.  Each lane's words pass
  // through its own LDS ring of kDecRing slots (words rd..wr-1, one slot
  // column per thread, so the ring accesses of a wave are bank-conflict free).
  // The ring is topped up in blocks of four words at group boundaries from
  // global loads issued one block ahead, so decoding waits on LDS only.
  // Indexes past the payload are clamped to its last word (those bits are
  // never part of a valid codeword).
  const uint64_t wlast = nwords - 1;
  uint32_t* R = ring + threadIdx.x;
  auto gw = [&](uint64_t i) { return words[i < wlast ? i : wlast]; };
  uint64_t rd = pos >> 5;
  uint64_t wr = rd;
  uint64_t buf;
  int have;
  uint32_t pre;
  {
    uint32_t x[12];
#pragma unroll
    for (int q = 0; q < 12; q++) x[q] = gw(wr + q);
#pragma unroll
    for (int q = 0; q < 12; q++) R[((wr + q) & (kDecRing - 1)) * 256] = x[q];
    wr += 12;
    const uint32_t skip = (uint32_t)(pos & 31);
    buf = ((uint64_t)x[0] << 32) << skip;
    have = 32 - (int)skip;
    rd++;
    pre = x[1];
  }
  uint32_t st0 = gw(wr), st1 = gw(wr + 1), st2 = gw(wr + 2), st3 = gw(wr + 3);
  // a group of eight symbols moves at most eight words into the buffer and
  // reads `pre` one word further: nine words must be in the ring
  auto top_up = [&]() {
    if (wr + 4 <= rd + kDecRing) {
      R[(wr & (kDecRing - 1)) * 256] = st0;
      R[((wr + 1) & (kDecRing - 1)) * 256] = st1;
      R[((wr + 2) & (kDecRing - 1)) * 256] = st2;
      R[((wr + 3) & (kDecRing - 1)) * 256] = st3;
      wr += 4;
      st0 = gw(wr), st1 = gw(wr + 1), st2 = gw(wr + 2), st3 = gw(wr + 3);
    }
    while (wr < rd + 9) {
      R[(wr & (kDecRing - 1)) * 256] = st0;
      R[((wr + 1) & (kDecRing - 1)) * 256] = st1;
      R[((wr + 2) & (kDecRing - 1)) * 256] = st2;
      R[((wr + 3) & (kDecRing - 1)) * 256] = st3;
      wr += 4;
      st0 = gw(wr), st1 = gw(wr + 1), st2 = gw(wr + 2), st3 = gw(wr + 3);
    }
  };
  uint32_t zeros = 0;
  bool bad = false;
  const uint32_t cnt_all = (uint32_t)(end - beg);
  // Full groups of eight codes: no per-symbol count checks (an invalid
  // codeword consumes one bit and marks the chunk bad; the bit count check at
  // the end catches the rest).  Chunks start at multiples of 64 symbols, so
  // every group is one 16-byte store.
  const uint32_t ngroups = cnt_all / 8;
  // the chunk is the slab c0 of brick b: its codes with c2 = 0 start every
  // fourth group (c1 = group / 4) and are contiguous in the compact array
  uint64_t f2base = 0;
  unsigned __int128 f2acc = 0;
  if (a.f2code) {
    const uint32_t b = (uint32_t)(k >> 5), c0 = (uint32_t)(k & 31);
    const uint32_t b2 = b % a.nbk2, b01 = b / a.nbk2;
    const uint32_t b1 = b01 % a.nbk1, b0 = b01 / a.nbk1;
    f2base = (uint64_t)b2 * a.f2_plane + (uint64_t)(b0 * 32 + c0) * a.f2_n1 + b1 * 32;
  }
  // eight symbols decoded into one 16-byte group
  auto group = [&]() {
    uint32_t pk[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (uint32_t t = 0; t < 8; t++) {
      // refill without a branch: the ring read of the next word is issued at
      // every step, beside the table lookup
      const bool need = have < 32;
      buf |= need ? ((uint64_t)pre << 32) >> (have & 31) : 0ull;
      have += need ? 32 : 0;
      rd += need ? 1 : 0;
      pre = R[(rd & (kDecRing - 1)) * 256];
      uint32_t L;
      uint32_t sym = decode_one<MODE>(a, lut, slong, sorted, subl, sbase, (uint32_t)(buf >> 32), L);
      bad |= L == 0;
      L = L ? L : 1u;
      zeros += sym == 0;
      buf <<= L;
      have -= (int)L;
      pos += L;
      pk[t >> 1] |= sym << ((t & 1) * 16);
    }
    return make_uint4(pk[0], pk[1], pk[2], pk[3]);
  };
  auto face2 = [&](uint32_t gi, uint32_t first) {
    if (a.f2code && (gi & 3) == 0) {
      // eight of them (c1 = 8m .. 8m + 7) collected, then one 16-byte store
      f2acc = (f2acc >> 16) | ((unsigned __int128)(first & 0xFFFFu) << 112);
      if ((gi & 31) == 28)
        *reinterpret_cast<unsigned __int128*>(a.f2code + f2base + (gi >> 2) - 7) = f2acc;
    }
  };
  // Whole 128-byte lines of codes are held in registers and stored together:
  // the 64 lanes of a wave write 64 chunks 2 KiB apart, and a line written a
  // group at a time leaves the cache partly filled between its stores.
  const uint32_t nlines = ngroups / 8;
  for (uint32_t li = 0; li < nlines; li++) {
    uint4 l0, l1, l2, l3, l4, l5, l6, l7;
#pragma unroll 1
    for (uint32_t g = 0; g < 8; g++) {
      top_up();
      const uint4 v = group();
      face2(li * 8 + g, v.x);
      l0 = l1, l1 = l2, l2 = l3, l3 = l4, l4 = l5, l5 = l6, l6 = l7, l7 = v;
    }
    uint4* dst = reinterpret_cast<uint4*>(code + beg + 64 * li);
    dst[0] = l0, dst[1] = l1, dst[2] = l2, dst[3] = l3;
    dst[4] = l4, dst[5] = l5, dst[6] = l6, dst[7] = l7;
  }
  for (uint32_t gi = nlines * 8; gi < ngroups; gi++) {
    top_up();
    const uint4 v = group();
    *reinterpret_cast<uint4*>(code + beg + 8 * gi) = v;
    face2(gi, v.x);
  }
  // the tail of the last chunk of the field (fewer than eight symbols)
  top_up();
  for (uint32_t t = ngroups * 8; t < cnt_all && !bad; t++) {
    if (have < 32) {
      buf |= ((uint64_t)pre << 32) >> have;
      have += 32;
      rd++;
      pre = R[(rd & (kDecRing - 1)) * 256];
    }
    uint32_t L;
    const uint32_t sym = decode_one<MODE>(a, lut, slong, sorted, subl, sbase, (uint32_t)(buf >> 32), L);
    if (!L) {
      bad = true;
      break;
    }
    zeros += sym == 0;
    buf <<= L;
    have -= (int)L;
    pos += L;
    code[beg + t] = (uint16_t)sym;
  }
  if (bad || pos != stop) atomicOr(status, 1);
  czero[k] = zeros;
}

hipError_t launch_decode2(const DecodeArgs& a, const uint32_t* words, const uint16_t* cbits,
                          uint64_t* tflags, const uint32_t* lut, const uint16_t* sorted,
                          const uint32_t* sub, uint16_t* code, uint32_t* czero, int* status,
                          hipStream_t st)
{
  if (!a.nch) return hipSuccess;
  const dim3 grid((unsigned)((a.nch + 255) / 256)), block(256);
  // built second-level tables rewrite first-level entries: mode 2 reads them
  if (a.n_sub && a.n_sub <= kDecSub)
    hipLaunchKernelGGL(decode2_kernel<2>, grid, block, 0, st, a, words, cbits, tflags, lut, sorted, sub,
                       code, czero, status);
  else if (a.n_long <= kDecLong)
    hipLaunchKernelGGL(decode2_kernel<0>, grid, block, 0, st, a, words, cbits, tflags, lut, sorted, sub,
                       code, czero, status);
  else
    hipLaunchKernelGGL(decode2_kernel<1>, grid, block, 0, st, a, words, cbits, tflags, lut, sorted, sub,
                       code, czero, status);
  return hipGetLastError();
}

template hipError_t launch_scatter_unpred2<float>(const uint16_t*, uint64_t, uint32_t,
                                                  const uint32_t*, const uint64_t*, const float*,
                                                  uint64_t, float*, int*, const Geom&, hipStream_t);
template hipError_t launch_scatter_unpred2<double>(const uint16_t*, uint64_t, uint32_t,
                                                   const uint32_t*, const uint64_t*, const double*,
                                                   uint64_t, double*, int*, const Geom&, hipStream_t);
template hipError_t launch_gather_unpred<float>(const uint16_t*, uint64_t, uint32_t, uint32_t*,
                                                uint64_t*, uint64_t*, const float*, float*,
                                                const Geom&, hipStream_t);
template hipError_t launch_gather_unpred<double>(const uint16_t*, uint64_t, uint32_t, uint32_t*,
                                                 uint64_t*, uint64_t*, const double*, double*,
                                                 const Geom&, hipStream_t);

}  // namespace hpez
