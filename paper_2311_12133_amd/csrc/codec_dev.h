// codec_dev.h -- declarations of the single-pass encoder and the decoder.
#pragma once

#include "hpez_internal.h"

namespace hpez {

constexpr uint32_t kEncTab = 8192;   // codebook entries held in LDS by the encoder
constexpr uint32_t kEncWords = 1026; // LDS words per chunk (1024 symbols x 32 bits + 2)
constexpr uint32_t kDecLong = 8192;  // codes longer than the decode table kept in LDS
// second-level decode table entries (LDS; with the first level, the symbols of
// the long codes and the input rings, two decoding work-groups still fit in
// one CU's 160 KiB)
constexpr uint32_t kDecSub = 8064;
// index bits of one second-level table at most: codes longer than kLutBits +
// kDecSubBits are found by the canonical limits instead
constexpr int kDecSubBits = 9;

struct EncodeArgs {
  uint64_t n;        // symbols
  uint64_t nch;      // chunks
  uint32_t chunk;    // symbols per chunk (64..1024)
  uint32_t smin;     // first symbol of the packed table
  uint32_t ntab;     // entries of the packed table (smax - smin + 1)
  int32_t lds_tab;   // the packed table fits in LDS
  int32_t packed_ok; // every symbol has a packed entry (below)
  int32_t pad;
  // Packed entry: codeword << 6 | length for codewords of at most 26 bits;
  // longer ones (up to 32 bits) are escaped as index << 6 | 63 into ltab,
  // whose entries are codeword << 6 | length (nullptr when there are none).
  const uint64_t* ltab;
};

// Canonical-code decoding state.  A 32-bit window w (next bits, first bit in
// the most significant position) starts a codeword of length l iff
// lim[l-1] <= w < lim[l]; that codeword's symbol is sorted[base[l] + (w >> (32 - l))].
struct DecodeArgs {
  uint64_t n;        // symbols
  uint64_t nch;      // chunks
  uint64_t nbits;    // payload bits
  uint32_t chunk;
  uint32_t long_first;       // index in sorted[] of the first code longer than kLutBits
  uint32_t n_long;           // number of such codes (held in LDS when <= kDecLong)
  uint32_t n_sub;            // second-level table entries (0: none; long codes by limits)
  // optional: codes of the points on the face planes x2 = 0 (mod 32) also go to
  // a compact array (every brick full, chunks of 1024 = one 32 x 32 slab of a
  // brick): index b2 * f2_plane + x0 * f2_n1 + x1; null when not used
  uint16_t* f2code;
  uint64_t f2_plane;
  uint32_t f2_n1, nbk1, nbk2;
  uint64_t lim[kLmax + 1];   // lim[l] = (first code of length l + count) << (32 - l)
  uint32_t base[kLmax + 1];  // offset of length l in sorted[] minus its first code (mod 2^32)
};

hipError_t launch_encode1(const EncodeArgs& a, const uint16_t* code, uint32_t* words,
                          uint16_t* out_cb, uint64_t* flags, uint32_t* ticket,
                          const uint32_t* packed, const uint8_t* len, const uint32_t* cw,
                          hipStream_t st);
// Up to kMaxSegs copies or zero fills in one launch: segment i writes n bytes
// at dst from src, or zeros when src is null.  dst and src 8-byte aligned.
constexpr int kMaxSegs = 8;
struct ByteSeg {
  uint8_t* dst;
  const uint8_t* src;
  uint64_t n;
};
struct ByteSegs {
  ByteSeg s[kMaxSegs];
  int count;
};
hipError_t launch_byte_segs(const ByteSegs& a, hipStream_t st);

// per-chunk counts of code 0 and their exclusive scan (zoff[nch] = total)
hipError_t launch_count_zeros(const uint16_t* code, uint64_t n, uint32_t chunk, uint32_t* czero,
                              uint64_t* zoff, uint64_t* tmp, hipStream_t st);
// verbatim values (code 0) gathered in stream order; counts zeros first
template <typename T>
hipError_t launch_gather_unpred(const uint16_t* code, uint64_t n, uint32_t chunk, uint32_t* czero,
                                uint64_t* zoff, uint64_t* tmp, const T* X, T* unpred, const Geom& g,
                                hipStream_t st);
// verbatim values scattered from stream order into W (decompress); a rank at or
// beyond n_unpred sets *d_status
template <typename T>
hipError_t launch_scatter_unpred2(const uint16_t* code, uint64_t n, uint32_t chunk,
                                  const uint32_t* czero, const uint64_t* zoff, const T* unpred,
                                  uint64_t n_unpred, T* W, int* d_status, const Geom& g,
                                  hipStream_t st);
// second-level tables of the codes longer than kLutBits: every kLutBits-bit
// prefix that starts such codes gets a table indexed by the next
// k = min(lmax - kLutBits, kDecSubBits) bits (lmax: its longest code), and its
// first-level entry becomes (table offset << 8) | 0x80 | k.  Entries of codes
// longer than kLutBits + k stay 0 (found by the canonical limits).  Returns the
// entries used, or 0 (tables not built, first level unchanged) when they would
// exceed cap.
uint32_t decode_subtables(const uint8_t* len, uint32_t lo, uint32_t hi, uint32_t* lut,
                          uint32_t* sub, uint32_t cap);

// cbits: the stream's per-chunk bit counts; tflags: one word per 256 chunks,
// zeroed; status[0] is set on a decoding error, status[1] (zeroed) is the
// work-groups' ticket counter
hipError_t launch_decode2(const DecodeArgs& a, const uint32_t* words, const uint16_t* cbits,
                          uint64_t* tflags, const uint32_t* lut, const uint16_t* sorted,
                          const uint32_t* sub, uint16_t* code, uint32_t* czero, int* status,
                          hipStream_t st);

}  // namespace hpez
