// Contraction entry point that allocates nothing on the device, for callers
// that cannot call hipMalloc (code under HIP graph capture of their own,
// tight serving loops, harnesses that forbid it).  The workspace of the call
// (slice ids, closed bits, leaf jobs, flags, scales and the intermediate
// arena) lives in one file-scope device array; each GPU the library runs on
// holds its own copy of it until the process ends.
#include <mutex>

#include "executor.h"

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;  // 256 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array.  The array's name is a
// host-side stand-in in host code; its device address is looked up once per
// device, with that device current, and kept.
void* scratch_address() {
  int dev = -1;
  rqc::hip_check(hipGetDevice(&dev), "current device");
  if (dev < 0 || dev >= kMaxDevices) throw rqc::Error{RQC_EUNSUPPORTED, "device ordinal above 63"};
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    rqc::hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "scratch address");
    if (!ptr) throw rqc::Error{RQC_EDEVICE, "scratch address is NULL"};
    g_scratch[dev] = ptr;
  }
  return g_scratch[dev];
}

}  // namespace

extern "C" {

rqc_status rqc_contract_noalloc(rqc_plan* p, const uint64_t* slice_ids, uint64_t n_ids,
                                const uint8_t* closed_bits, uint64_t n_batch, int32_t prec,
                                double* out, double* per_slice, rqc_stream stream) {
  try {
    if (!p) throw rqc::Error{RQC_EINVAL, "NULL plan"};
    if (prec != RQC_F32 && prec != RQC_F16 && prec != RQC_BF16) throw rqc::Error{RQC_EINVAL, "bad precision"};
    if (n_batch == 0) throw rqc::Error{RQC_EINVAL, "n_batch must be positive"};
    // The smallest grouping (one slice and one bitstring at a time) must fit.
    const uint64_t ids = slice_ids ? n_ids : (uint64_t(1) << p->pd.sliced.size());
    const rqc::GroupLayout& L1 = rqc::group_layout(p, prec, 1, 1);
    const int64_t need = rqc::ws_layout(p, L1, ids, n_batch).total;
    if (need > (int64_t)kScratchBytes)
      throw rqc::Error{RQC_EHBM, "call needs at least " + std::to_string(need) +
                                     " workspace bytes, above the 268435456-byte static scratch "
                                     "of rqc_contract_noalloc"};
    void* ws = scratch_address();
    rqc::contract(p, slice_ids, n_ids, closed_bits, n_batch, prec, ws, kScratchBytes, out, per_slice,
                  static_cast<hipStream_t>(stream), p->pending, /*direct=*/true);
    return RQC_OK;
  } catch (const rqc::Error& e) {
    rqc::set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    rqc::set_error("host allocation failed");
    return RQC_ENOMEM;
  } catch (const std::exception& e) {
    rqc::set_error(e.what());
    return RQC_EINVAL;
  }
}

uint64_t rqc_contract_noalloc_scratch_bytes(void) { return kScratchBytes; }

}  // extern "C"
