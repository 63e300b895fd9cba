// codec_dev.h -- declarations of the single-pass encoder and the decoder.
#pragma once

#include "hpez_internal.h"

namespace hpez {

constexpr uint32_t kEncTab = 8192;   // codebook entries held in LDS by the encoder
constexpr uint32_t kEncWords = 1026; // LDS words per chunk (1024 symbols x 32 bits + 2)

struct EncodeArgs {
  uint64_t n;        // symbols
  uint64_t nch;      // chunks
  uint32_t chunk;    // symbols per chunk (64..1024)
  uint32_t smin;     // first symbol of the packed table
  uint32_t ntab;     // entries of the packed table (smax - smin + 1)
  int32_t lds_tab;   // the packed table fits in LDS
  int32_t packed_ok; // every codeword fits the packed entry (length <= 26)
  int32_t pad;
};

struct DecodeArgs {
  uint64_t n;
  uint64_t nch;
  uint64_t nbits;
  uint32_t chunk;
  uint32_t pad;
};

hipError_t launch_encode1(const EncodeArgs& a, const uint16_t* code, uint32_t* words,
                          uint16_t* out_cb, uint64_t* flags, uint32_t* ticket,
                          const uint32_t* packed, const uint8_t* len, const uint32_t* cw,
                          hipStream_t st);
template <typename T>
hipError_t launch_gather_unpred(const uint16_t* code, uint64_t n, uint32_t chunk, uint32_t* czero,
                                uint64_t* zoff, uint64_t* tmp, const T* X, T* unpred, const Geom& g,
                                hipStream_t st);
hipError_t launch_decode2(const DecodeArgs& a, const uint32_t* words, const uint64_t* bit_off,
                          const uint32_t* lut, const uint32_t* first, const uint32_t* count,
                          const uint32_t* offset, const uint16_t* sorted, uint16_t* code,
                          uint32_t* czero, int* status, hipStream_t st);

}  // namespace hpez
