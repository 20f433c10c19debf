// The allocation-free form of lbm_step (include/lbm.h, lbm_step_static): the caller
// passes the two state buffers and receives the force rows on the host; every other
// device buffer a step reads or writes (pull codes, strip slots, inlet profile, body
// motion, force partials, box-sweep partials, force rows) lives in `scratch`, a
// file-scope device array of fixed size.  Each GPU holds its own copy of the array from
// the first call on it until the process ends; its address on each device is looked up
// once, with that device current, and only that address is handed to kernels and
// copies.  The array keeps the last call's contents: every byte a call reads is written
// by the same call first.  Calls that overlap on one GPU race for the array.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "handle.h"
#include "kernels.h"
#include "lbm.h"
#include "plan.h"
#include "trace.h"

// The static scratch of every GPU (its host-side name is a stand-in, never a device
// address: host code uses the address hipGetSymbolAddress gives on each device).
static __device__ __align__(256) unsigned char scratch[size_t(LBM_STATIC_SCRATCH_BYTES)];

namespace {

constexpr size_t kScratchBytes = size_t(LBM_STATIC_SCRATCH_BYTES);
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Device address of `scratch` on the current device, looked up on the first call there.
hipError_t scratch_on_current_device(void** out, std::string& why) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    why = "hipGetDevice";
    return e;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    why = "device index beyond the static scratch table";
    return hipErrorInvalidDevice;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      why = "hipGetSymbolAddress(scratch)";
      return e != hipSuccess ? e : hipErrorInvalidSymbol;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

int lbm_step_static(lbm_t* h, void* buf0, void* buf1, size_t buf_bytes, int32_t n,
                    uint32_t force_scheme, double* forces, int64_t cap, void* hip_stream) {
  using namespace lbm;
  TraceRange range("lbm_step_static");
  if (!h) return LBM_EINVAL;
  if (n < 0) return h->fail(LBM_EINVAL, "n must be >= 0");
  if (force_scheme & ~LBM_FORCE_ALL) return h->fail(LBM_EINVAL, "unknown force scheme bits");
  if (h->g.precision == LBM_FP32SR)
    return h->fail(LBM_EINVAL, "the stochastically rounded storage needs the handle's step count; "
                               "use lbm_step");
  if (!buf0 || !buf1 || buf0 == buf1 || reinterpret_cast<uintptr_t>(buf0) % 256 ||
      reinterpret_cast<uintptr_t>(buf1) % 256)
    return h->fail(LBM_EINVAL, "two distinct 256-byte aligned state buffers are needed");
  if (buf_bytes < h->buf_bytes())
    return h->fail(LBM_ENOMEM, "state buffers smaller than one state of the handle");
  const bool want = force_scheme != 0 && n > 0;
  if (want && (!forces || cap < n))
    return h->fail(LBM_EINVAL, "force output holds fewer rows than steps");
  if (n == 0) return LBM_OK;
  const Plan& p = h->plan;
  // Layout of the scratch array for this call.
  size_t off = 0;
  const size_t off_node = off;
  off = align256(off + p.node.size() * sizeof(uint32_t));
  const size_t off_slot = off;
  off = align256(off + p.strip_slot.size() * sizeof(int32_t));
  const size_t off_uin = off;
  off = align256(off + size_t(p.ny) * sizeof(double));
  const size_t off_mot = off;
  off = align256(off + sizeof(BodyMotion));
  const size_t off_part = off;
  const size_t part = align256(h->part_doubles() * sizeof(double));
  off += 2 * part;
  const size_t off_jpart = off;
  off = align256(off + size_t(h->njblocks) * 2 * sizeof(double));
  const size_t off_ring = off;
  if (want) off = align256(off + size_t(n) * kRingRow * sizeof(double));
  if (off > kScratchBytes)
    return h->fail(LBM_ENOMEM, "the grid and step count need " + std::to_string(off) +
                                   " bytes of static scratch; the limit is " +
                                   std::to_string(kScratchBytes));
  void* sp = nullptr;
  std::string why;
  hipError_t e = scratch_on_current_device(&sp, why);
  if (e != hipSuccess) return h->hip_fail(e, why.c_str());
  char* s = static_cast<char*>(sp);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  e = hipMemcpyAsync(s + off_node, p.node.data(), p.node.size() * sizeof(uint32_t),
                     hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s + off_slot, p.strip_slot.data(), p.strip_slot.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s + off_uin, h->uin.data(), size_t(p.ny) * sizeof(double),
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess && h->motion.moving)
    e = hipMemcpyAsync(s + off_mot, &h->motion, sizeof(BodyMotion), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return h->hip_fail(e, "upload tables to the static scratch");
  DevTables t{};
  t.node = reinterpret_cast<const uint32_t*>(s + off_node);
  t.strip_slot = reinterpret_cast<const int32_t*>(s + off_slot);
  t.uin = reinterpret_cast<const double*>(s + off_uin);
  t.motion = h->motion.moving ? reinterpret_cast<const BodyMotion*>(s + off_mot) : nullptr;
  t.part[0] = reinterpret_cast<double*>(s + off_part);
  t.part[1] = reinterpret_cast<double*>(s + off_part + part);
  t.jpart = reinterpret_cast<double*>(s + off_jpart);
  double* ring = want ? reinterpret_cast<double*>(s + off_ring) : nullptr;
  const int rc = enqueue_pingpong(h, t, buf0, buf1, st, n, ring);
  if (rc != LBM_OK) return rc;
  if (!want) return LBM_OK;
  std::vector<double> rows(size_t(n) * kRingRow);
  e = hipMemcpyAsync(rows.data(), ring, rows.size() * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return h->hip_fail(e, "download force rows");
  bool finite = true;
  for (int32_t k = 0; k < n; ++k)
    finite = row_forces(&rows[size_t(k) * kRingRow], force_scheme, p.has_box,
                        forces + int64_t(k) * 2 * kSchemes) && finite;
  if (!finite) return h->fail(LBM_ENONFINITE, "a recorded force is not finite");
  return LBM_OK;
}

}  // extern "C"
