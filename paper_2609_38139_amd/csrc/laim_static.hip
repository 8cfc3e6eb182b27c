// laim_static.hip -- laim_decode_rounds_static: the decode call for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid allocation). Its scratch -- the shot
// queue of the resident form, or the message buffers of the stream form --
// is a file-scope device array of fixed size instead of a workspace
// argument; everything else is laim_decode_rounds.
#include <hip/hip_runtime.h>

#include <mutex>

#include "laim_internal.h"

// The scratch array. Each device the library runs on holds its own copy, at
// its own address, until the process ends. In host code this name is only a
// stand-in for the symbol: its device address comes from
// hipGetSymbolAddress (scratch_address below), and only that address is
// passed to kernels.
static __device__ __align__(256) unsigned char scratch[LAIM_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device, once looked up

struct DeviceGuard {
  int prev = 0;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    (void)hipGetDevice(&prev);
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() { (void)hipSetDevice(prev); }
};

// The device address of `scratch` on `device`, looked up on the first call
// for that device with the device current.
laim_status scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) {
    laim::set_error("device %d is beyond the %d devices the static scratch supports", device,
                    kMaxDevices);
    return LAIM_EUNSUP;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    DeviceGuard g(device);
    if (!g.ok) {
      laim::set_error("cannot make device %d current", device);
      return LAIM_EHIP;
    }
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return laim::hip_fail(e, "looking up the static scratch");
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return LAIM_OK;
}

}  // namespace

extern "C" laim_status laim_decode_rounds_static(const laim_code* code,
                                                 const laim_decode_params* params,
                                                 const uint8_t* e0, uint64_t shot0, int32_t nshots,
                                                 uint8_t* z_out, uint8_t* s_out, int32_t* tclr_out,
                                                 float* L_out, int32_t* sweeps_out,
                                                 uint8_t* fail_out, int32_t form,
                                                 laim_stream stream) {
  if (!code || !params || nshots < 0) {
    laim::set_error("laim_decode_rounds_static: bad arguments");
    return LAIM_EINVAL;
  }
  if (nshots > 0) {
    // laim_workspace_bytes is 0 for arguments decode_common rejects below
    const size_t need = laim_workspace_bytes(code, params, nshots, form);
    if (need > (size_t)LAIM_STATIC_SCRATCH_BYTES) {
      laim::set_error("this call needs %zu bytes of scratch; the static scratch holds %zu (decode "
                      "fewer shots per call, or use the resident form)",
                      need, (size_t)LAIM_STATIC_SCRATCH_BYTES);
      return LAIM_ENOMEM;
    }
  }
  void* ws = nullptr;
  laim_status st = scratch_address(code->device, &ws);
  if (st != LAIM_OK) return st;
  return laim::decode_common(code, params, e0, shot0, nshots, ws, LAIM_STATIC_SCRATCH_BYTES, z_out,
                             s_out, tclr_out, L_out, sweeps_out, fail_out, form, nullptr, stream);
}
