// Forward pass whose launch scratch lives in a fixed file-scope device array,
// for callers that cannot allocate device memory at call time (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The array is reached through the address hipGetSymbolAddress returns on
// each device (the array's name in host code is a host-side stand-in, not a
// device address).  The plan's uploaded tables (entries, runs, groups) are
// read as with cm_contacts_fwd; everything the launches write besides the
// caller's output records -- survivor bitmasks and counts, offsets, per-entry
// filtered sums, the tile counter and the blend partials -- goes to the array.
#include <mutex>

#include "runtime.h"

namespace cm {

constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch` per device
}  // namespace

// Looks up the array's device address on `device` (current) once.  Called by
// cm_init for every context on a device.
hipError_t static_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device] != nullptr) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

static void* static_scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

// Bytes of launch scratch a forward pass over the plan needs; with base set,
// points the launch arguments at their parts of it.
static size_t forward_scratch(const cm_plan* pl, char* b, FwdArgs* a) {
  const PlanSizes z = layout_sizes(pl);  // the batch's sizes, or a reserved plan's capacity
  const int64_t W = std::max<int64_t>(z.W, 1);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t r = off; off = align_up(off + bytes, 256); return r; };
  const size_t o_bits = take(8 * size_t(W));
  const size_t o_nsurv = take(4 * size_t(z.E));
  const size_t o_wpre = take(4 * size_t(W));
  const size_t o_soff = take(8 * size_t(z.E + 1));
  const size_t o_ntr = take(4 * size_t(z.R));
  const size_t o_npart = take(4 * size_t(z.E));
  const size_t o_poff = take(8 * size_t(z.E + 1));
  const size_t o_filt = take(16 * size_t(z.E));
  const size_t o_toff = take(8 * size_t(z.R + 1));
  const size_t o_bsum = take(8 * size_t(z.nb + 1));
  const size_t o_cnt = take(256);
  const size_t o_part = take(4 * size_t(kStride) * size_t(W + z.E));
  if (b != nullptr) {
    a->bits = reinterpret_cast<uint64_t*>(b + o_bits);
    a->nsurv = reinterpret_cast<int32_t*>(b + o_nsurv);
    a->wpre = reinterpret_cast<int32_t*>(b + o_wpre);
    a->surv_off = reinterpret_cast<int64_t*>(b + o_soff);
    a->ntr = reinterpret_cast<int32_t*>(b + o_ntr);
    a->npart = reinterpret_cast<int32_t*>(b + o_npart);
    a->part_off = reinterpret_cast<int64_t*>(b + o_poff);
    a->filt = reinterpret_cast<F4*>(b + o_filt);
    a->tile_off = reinterpret_cast<int64_t*>(b + o_toff);
    a->bsum = reinterpret_cast<int64_t*>(b + o_bsum);
    a->counter = reinterpret_cast<uint32_t*>(b + o_cnt);
    a->partials = reinterpret_cast<float*>(b + o_part);
  }
  return off;
}

}  // namespace cm

extern "C" cm_status cm_contacts_fwd_noalloc(cm_context* ctx, cm_plan* pl, const cm_query* q, cm_groups out,
                                             void* stream) {
  using namespace cm;
  if (!ctx || !pl || pl->ctx != ctx || !q) return fail(ctx, CM_E_INVALID, "bad arguments");
  if (!out.p || !out.n || !out.d || !out.q || !out.W || !out.logZ) return fail(ctx, CM_E_INVALID, "null output");
  const size_t need = forward_scratch(pl, nullptr, nullptr);
  if (need > kStaticScratchBytes)
    return fail(ctx, CM_E_INVALID,
                "batch needs " + std::to_string(need) + " bytes of launch scratch; the fixed array holds " +
                    std::to_string(kStaticScratchBytes) + " (split the batch into smaller plans)");
  char* base = static_cast<char*>(static_scratch_ptr(ctx->device));
  if (base == nullptr) return fail(ctx, CM_E_HIP, "fixed scratch array not set up on this device");
  FwdArgs a = fwd_args(ctx, pl, q, out, nullptr);
  forward_scratch(pl, base, &a);
  a.ev = nullptr;    // no timing events
  a.work = nullptr;  // no work counters
  a.tape = nullptr;
  a.tape_tiles = 0;
  const hipError_t e = launch_forward(a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(ctx, e, "forward launch (fixed scratch)");
  return CM_OK;
}
