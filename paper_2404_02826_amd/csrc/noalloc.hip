// noalloc.hip -- bbx_compress_static: bbx_compress with its workspace in a
// file-scope device array, for callers that cannot allocate device memory.
//
// The array (kStaticScratch bytes) exists once per device that the library
// runs on and lives until the process ends.  Host code never passes the
// array's name to a kernel: on the first call on a device, with that device
// current, hipGetSymbolAddress gives the array's device address, which is
// kept per device and passed as the workspace.  Every call on a device uses
// the same memory, so calls that overlap on one device race; bbx_compress
// initialises every part of its workspace it reads, so nothing carries over
// from the previous call.
#include <mutex>
#include <string>

#include "bbx_internal.h"

namespace bbx {

constexpr size_t kStaticScratch = 64ull << 20;  // 64 MiB
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kStaticScratch];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// Device address of this device's scratch array (looked up once per device).
static bbx_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(BBX_EHIP, hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return set_error(BBX_EUNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(BBX_EHIP, (std::string("scratch address lookup failed: ") + hipGetErrorString(e)).c_str());
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return BBX_OK;
}

}  // namespace bbx

extern "C" {

size_t bbx_compress_static_limit(void) { return bbx::kStaticScratch; }

bbx_status bbx_compress_static(const void* d_pos, uint64_t n, uint32_t dims, bbx_dtype dtype,
                               double eb, const bbx_params* params, void* d_out, size_t out_cap,
                               size_t* h_out_size, uint64_t* d_size, uint32_t* d_status,
                               uint32_t* d_perm, hipStream_t stream) {
  const size_t need = bbx_compress_workspace_size(n, dims, dtype, params);
  if (need == 0) return bbx_compress(d_pos, n, dims, dtype, eb, params, d_out, out_cap, h_out_size,
                                     d_size, d_status, d_perm, nullptr, 0, stream);  // argument error
  if (need > bbx::kStaticScratch)
    return bbx::set_error(BBX_ENOMEM, ("set needs " + std::to_string(need) +
                                       " bytes of workspace, above the 64 MiB static scratch").c_str());
  void* ws = nullptr;
  bbx_status st = bbx::scratch_address(&ws);
  if (st != BBX_OK) return st;
  return bbx_compress(d_pos, n, dims, dtype, eb, params, d_out, out_cap, h_out_size, d_size,
                      d_status, d_perm, ws, bbx::kStaticScratch, stream);
}

}  // extern "C"
