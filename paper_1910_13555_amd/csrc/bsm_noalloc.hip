// Allocation-free execute (bsm_plan_execute_noalloc): the numeric phase of a
// plan with every device buffer it needs beyond the caller's inputs and
// outputs taken from one fixed array in the library's own device memory, for
// callers that cannot allocate (HIP graph capture, serving loops).
//
// Of the numeric phase's paths only split precision needs scratch: the
// bfloat16 piece arrays of both operands, written by the split pass and read
// by the numeric kernels.  They go to `scratch`, one copy per device, whose
// address each device reports once through hipGetSymbolAddress (the array's
// name in host code is not a device address).  The split pass rewrites the
// whole used part of the array, zero tails included, on every call, so
// nothing has to be cleared in between.  Calls on one device share the
// array: calls whose work overlaps on a device (different streams) race.
#include "bsm_host.h"

#include <mutex>

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;   // 256 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (the device is current).
void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) fail(BSM_E_UNSUPPORTED, "device %d beyond %d", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch address");
    if (!p) fail(BSM_E_DEVICE, "no device address for the scratch array");
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

}  // namespace

extern "C" bsm_status bsm_plan_execute_noalloc(bsm_plan pl, double alpha, const double* a_vals,
                                               const double* b_vals, double beta, const double* c_in_vals,
                                               double* c_out_vals) {
  return guard([&] {
    if (!pl) fail(BSM_E_INVALID, "NULL plan");
    if (pl->ext && pl->ext->remaps())
      fail(BSM_E_UNSUPPORTED, "contraction plans that permute operands or the output need scratch of their size");
    if (split_scratch_bytes(pl) > kScratchBytes)
      fail(BSM_E_UNSUPPORTED, "split precision needs %zu bytes of piece arrays; the fixed scratch holds %zu",
           split_scratch_bytes(pl), kScratchBytes);
    set_device(pl->ctx);
    Scratch sc;
    sc.p = scratch_address(pl->ctx->device);
    sc.bytes = kScratchBytes;
    execute(pl, alpha, a_vals, b_vals, beta, c_in_vals, c_out_vals, &sc);
  });
}
