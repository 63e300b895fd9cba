// noalloc.hip -- hpez_decompress_noalloc: decompression whose device workspace
// is a static device array of the library instead of memory the library
// allocates, for callers that cannot allocate (code under graph capture,
// serving loops, harnesses that forbid hipMalloc).
//
// The array `scratch` is a file-scope __device__ variable, so every GPU the
// library runs on holds its own copy from module load until the process ends.
// In host code its name is only a stand-in: the device address of a GPU's
// copy comes from hipGetSymbolAddress, called once per device with that device
// current, and only that address reaches kernels and copies.  Calls on one
// GPU share its copy (the previous call's contents stay): the decompression
// clears what must start at zero itself, and calls that overlap on one GPU
// race.

#include <mutex>

#include "hpez_host.h"
#include "hpez_internal.h"

namespace hpez {
namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // 64 MiB per GPU

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

struct ScratchSlot {
  std::once_flag once;
  int rc = HPEZ_OK;
  void* ptr = nullptr;  // device address of this GPU's copy of scratch
};
ScratchSlot g_slot[kFixedDevices];

// the device address of `device`'s copy, looked up once with the device current
int scratch_of(int device, void** out)
{
  ScratchSlot& s = g_slot[device];
  std::call_once(s.once, [&] {
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (hipSetDevice(device) != hipSuccess) {
      s.rc = HPEZ_EDEVICE;
      return;
    }
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    s.rc = (e == hipSuccess && p) ? HPEZ_OK : HPEZ_EDEVICE;
    s.ptr = s.rc == HPEZ_OK ? p : nullptr;
    if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
  });
  *out = s.ptr;
  return s.rc;
}

}  // namespace
}  // namespace hpez

extern "C" {

int hpez_decompress_noalloc(int device, const void* d_in, uint64_t in_size, void* d_out,
                            uint64_t out_cap, hipStream_t stream)
{
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) return HPEZ_EDEVICE;
  if (device < 0 || device >= ndev || device >= hpez::kFixedDevices || !d_in || !d_out)
    return HPEZ_EINVAL;
  void* ws = nullptr;
  const int rc = hpez::scratch_of(device, &ws);
  if (rc) return rc;
  return hpez::decompress_fixed(device, ws, hpez::kScratchBytes, d_in, in_size, d_out, out_cap,
                                stream);
}

}  // extern "C"
