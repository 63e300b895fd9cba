// lossless_dev.h -- launchers of the lossless stage after Huffman coding
// (Sec. 4, step 5): zero-run tokens of a byte string, and their expansion.
//
// Tokens: a nonzero byte v is token v (1..255); a maximal run of k zero bytes
// is floor(k / kRunMax) tokens 255 + kRunMax, then token 255 + (k mod kRunMax)
// when that is not 0.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace hpez {

constexpr uint32_t kRunMax = 4096;
constexpr uint32_t kTokSyms = 256 + kRunMax;  // token alphabet [0, kTokSyms), 0 unused
constexpr uint64_t kLLTile = 4096;            // bytes per work-group of the byte passes

// per tile of kLLTile bytes: the count of nonzero bytes
hipError_t launch_ll_count(const uint8_t* b, uint64_t n, uint32_t* cnt, hipStream_t st);
// positions (in order) of the nonzero bytes; tile_off: exclusive scan of cnt
hipError_t launch_ll_compact(const uint8_t* b, uint64_t n, const uint64_t* tile_off,
                             uint32_t* pos, hipStream_t st);
// tcnt[j] for j in [0, n]: tokens of the zero run before nonzero byte j (the
// run after the last one for j = nnz) plus its literal; 0 for j > nnz.
// nnz: device count of nonzero bytes.
hipError_t launch_ll_tokcount(const uint32_t* pos, const uint64_t* nnz, uint64_t n,
                              uint32_t* tcnt, hipStream_t st);
// the tokens at toff[j] (exclusive scan of tcnt) and their histogram (hist:
// kTokSyms words, zeroed)
hipError_t launch_ll_tokens(const uint8_t* b, const uint32_t* pos, const uint64_t* nnz, uint64_t n,
                            const uint64_t* toff, uint16_t* tok, uint32_t* hist, hipStream_t st);
// bytes of each of ntok tokens (status[0] set for a token outside [1, 255 + kRunMax])
hipError_t launch_ll_toklen(const uint16_t* tok, uint64_t ntok, uint32_t* len, int* status,
                            hipStream_t st);
// literal bytes of the tokens at their offsets (off: exclusive scan of the
// token lengths) into the zeroed output of n bytes
hipError_t launch_ll_expand(const uint16_t* tok, uint64_t ntok, const uint64_t* off, uint8_t* out,
                            uint64_t n, int* status, hipStream_t st);

}  // namespace hpez
