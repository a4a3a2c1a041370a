// Selection of one round without any allocation: the priority threshold
// (all pending, exact top ceil(q n), sampled, or the round-robin block) and
// the 0/1 selection of every vertex, computed from caller device arrays into
// caller device arrays. The scratch the selection kernels need (control
// block, radix histograms, sampled keys, per-block partials) lives in one
// file-scope device array of fixed size; every call on a device uses that
// device's copy, so calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "daic_device.h"
#include "daic_internal.h"
#include "daic_kernels.h"

namespace daic {
namespace {

constexpr size_t kAlign = 256;
constexpr size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Layout of the scratch array. The per-vertex kernels use at most
// kMaxScanBlocks blocks whatever n is, so the size does not depend on n.
constexpr size_t kOffCtl = 0;
constexpr size_t kOffHist = align_up(kOffCtl + sizeof(Ctl));
constexpr size_t kOffKeys = align_up(kOffHist + (size_t)kRadixBins * kRadixCopies * 4);
constexpr size_t kOffTies = align_up(kOffKeys + (size_t)kMaxSamples * 8);
constexpr size_t kOffTieOff = align_up(kOffTies + (size_t)kMaxScanBlocks * 4);
constexpr size_t kOffPartR = align_up(kOffTieOff + ((size_t)kMaxScanBlocks + 1) * 8);
constexpr size_t kOffPartN = align_up(kOffPartR + (size_t)kMaxScanBlocks * 8);
constexpr size_t kScratchBytes = align_up(kOffPartN + (size_t)kMaxScanBlocks * 8);
static_assert(kScratchBytes <= 160 * 1024, "the selection scratch is documented as under 160 KiB");

__device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::once_flag g_scratch_once[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices] = {};

// The device address of this device's scratch array, looked up once per
// device with that device current (the array's name is a host-side stand-in
// and must not be passed to kernels).
daic_status scratch_of_current_device(uint8_t** out) {
  int dev = 0;
  DAIC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(DAIC_E_UNSUPPORTED, "device index %d beyond %d", dev, kMaxDevices);
  std::call_once(g_scratch_once[dev], [dev] {
    void* p = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? p : nullptr;
  });
  if (g_scratch_err[dev] != hipSuccess || !g_scratch_ptr[dev])
    return fail(DAIC_E_DEVICE, "hipGetSymbolAddress of the selection scratch failed: %s",
                hipGetErrorString(g_scratch_err[dev]));
  *out = static_cast<uint8_t*>(g_scratch_ptr[dev]);
  return DAIC_OK;
}

// The threshold key of the round as a double (0 when every pending vertex
// is taken), as daic_select_frontier reports it.
template <int ST>
__global__ void k_threshold_out(const Ctl* ctl, double* out) {
  if (ctl->sel_mode == 0) {
    *out = 0.0;
  } else if constexpr (ST == ST_F64 || ST == ST_F64MIN) {
    *out = __longlong_as_double((long long)ctl->tau);
  } else if constexpr (ST == ST_F32 || ST == ST_F32K) {
    *out = (double)__uint_as_float((uint32_t)ctl->tau);
  } else {
    *out = (double)ctl->tau;
  }
}

template <int ST, int G>
void enqueue_select(const KArgs& a, const daic_run_opts* o, uint64_t round, double* d_tau, hipStream_t s) {
  using Key = typename Tr<ST>::Key;
  const uint64_t n = a.n;
  hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(1), 0, s, a.ctl, 0.0, ~0ull);
  hipLaunchKernelGGL(k_residual<ST>, dim3(a.blocks), dim3(256), 0, s, a, 0);
  hipLaunchKernelGGL(k_residual_final<ST>, dim3(1), dim3(256), 0, s, a, 0, 0ull, 0ull, 0);
  hipLaunchKernelGGL(k_clear_done, dim3(1), dim3(1), 0, s, a.ctl);  // the selection runs on a finished state too
  if (o->sched == DAIC_SCHED_ALL) {
    hipLaunchKernelGGL(k_select_all, dim3(1), dim3(1), 0, s, a.ctl);
  } else if (o->sched == DAIC_SCHED_ROUND_ROBIN) {
    hipLaunchKernelGGL(k_select_rr, dim3(1), dim3(1), 0, s, a.ctl, (n + a.rr_chunk - 1) / a.rr_chunk);
  } else if (o->sched == DAIC_SCHED_TOPK_SAMPLED) {
    const uint32_t S = o->n_samples ? o->n_samples : kMaxSamples;
    const uint32_t rank = (uint32_t)std::max(1.0, std::ceil(o->priority_fraction * (double)S));
    hipLaunchKernelGGL(k_sample_keys<ST>, dim3((S + 255) / 256), dim3(256), 0, s, a, S, o->seed, round);
    hipLaunchKernelGGL(k_sample<ST>, dim3((S + 63) / 64), dim3(256), 0, s, a, S, rank);
  } else {
    uint64_t k = (uint64_t)std::ceil(o->priority_fraction * (double)n);
    if (k < 1) k = 1;
    const uint32_t hgrid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(1024, (n + 1023) / 1024));
    hipLaunchKernelGGL(k_topk_init, dim3(1), dim3(256), 0, s, a.ctl, a.rhist, k);
    for (int pass = 0; pass < radix_passes<Key>(); ++pass) {
      hipLaunchKernelGGL(k_radix_pass<ST>, dim3(hgrid), dim3(256), 0, s, a, pass);
      hipLaunchKernelGGL(k_radix_pick<ST>, dim3(1), dim3(256), 0, s, a, pass);
    }
    hipLaunchKernelGGL(k_tie_count<ST>, dim3(a.blocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_tie_scan, dim3(1), dim3(1024), 0, s, a);
  }
  // row offsets are not read by the selection-only claim
  hipLaunchKernelGGL((k_claim<ST, G, uint32_t, true>), dim3(a.blocks), dim3(256), 0, s, a);
  if (d_tau) hipLaunchKernelGGL(k_threshold_out<ST>, dim3(1), dim3(1), 0, s, a.ctl, d_tau);
}

}  // namespace
}  // namespace daic

using namespace daic;

extern "C" {

daic_status daic_select_frontier_noalloc(daic_op op, daic_dtype state, uint64_t n, const void* d_v, const void* d_dv,
                                         const daic_run_opts* o, uint64_t round, uint8_t* d_sel_out,
                                         double* d_threshold_out) {
  if (!o) return fail(DAIC_E_INVALID, "opts is null");
  if (n >= 0xFFFFFFFFull) return fail(DAIC_E_INVALID, "n must be below 2^32-1");
  if (n > 0 && (!d_v || !d_dv || !d_sel_out)) return fail(DAIC_E_INVALID, "null device array");
  if (!(o->priority_fraction > 0.0 && o->priority_fraction <= 1.0))
    return fail(DAIC_E_INVALID, "priority_fraction must be in (0, 1]");
  if (!(o->sched == DAIC_SCHED_ALL || o->sched == DAIC_SCHED_TOPK_EXACT || o->sched == DAIC_SCHED_TOPK_SAMPLED ||
        o->sched == DAIC_SCHED_ROUND_ROBIN))
    return fail(DAIC_E_UNSUPPORTED, "the no-allocation selection takes ALL, TOPK_EXACT, TOPK_SAMPLED or ROUND_ROBIN");
  if (o->sched == DAIC_SCHED_TOPK_SAMPLED && o->n_samples > kMaxSamples)
    return fail(DAIC_E_INVALID, "n_samples must be <= %u", kMaxSamples);
  int st;
  if (op == DAIC_SUM && state == DAIC_F64) st = ST_F64;
  else if (op == DAIC_SUM && state == DAIC_F32) st = ST_F32;
  else if (op == DAIC_SUM && state == DAIC_F32_KAHAN) st = ST_F32K;
  else if (op == DAIC_MIN && state == DAIC_U32) st = ST_U32;
  else if (op == DAIC_MIN && state == DAIC_F64) st = ST_F64MIN;
  else if (op == DAIC_MAX && state == DAIC_I32) st = ST_I32;
  else return fail(DAIC_E_UNSUPPORTED, "(+)/state combination not offered");
  if (n == 0) return DAIC_OK;
  uint8_t* base = nullptr;
  daic_status rc = scratch_of_current_device(&base);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(o->hip_stream);
  KArgs a{};
  a.ctl = reinterpret_cast<Ctl*>(base + kOffCtl);
  a.rhist = reinterpret_cast<uint32_t*>(base + kOffHist);
  a.skeys = reinterpret_cast<uint64_t*>(base + kOffKeys);
  a.blk_ties = reinterpret_cast<uint32_t*>(base + kOffTies);
  a.off_ties = reinterpret_cast<uint64_t*>(base + kOffTieOff);
  a.part_r = reinterpret_cast<double*>(base + kOffPartR);
  a.part_n = reinterpret_cast<uint64_t*>(base + kOffPartN);
  a.v = const_cast<void*>(d_v);  // read only: the claim runs in its selection-only form
  a.dv = const_cast<void*>(d_dv);
  a.n = n;
  const uint64_t blocks = std::min<uint64_t>(kMaxScanBlocks, (n + kScanBlock - 1) / kScanBlock);
  uint64_t per = (n + blocks - 1) / blocks;
  per = (per + kScanBlock - 1) / kScanBlock * kScanBlock;
  a.per_block = per;
  a.blocks = (uint32_t)((n + per - 1) / per);
  a.sel_out = d_sel_out;
  a.rr_chunk = std::max<uint64_t>(1, (uint64_t)std::ceil(o->priority_fraction * (double)n));
  switch (st) {
    case ST_F64: enqueue_select<ST_F64, DAIC_G_DEG_SCALE>(a, o, round, d_threshold_out, s); break;
    case ST_F32: enqueue_select<ST_F32, DAIC_G_DEG_SCALE>(a, o, round, d_threshold_out, s); break;
    case ST_F32K: enqueue_select<ST_F32K, DAIC_G_DEG_SCALE>(a, o, round, d_threshold_out, s); break;
    case ST_U32: enqueue_select<ST_U32, DAIC_G_EDGE_ADD>(a, o, round, d_threshold_out, s); break;
    case ST_F64MIN: enqueue_select<ST_F64MIN, DAIC_G_EDGE_ADD>(a, o, round, d_threshold_out, s); break;
    default: enqueue_select<ST_I32, DAIC_G_COPY>(a, o, round, d_threshold_out, s); break;
  }
  DAIC_HIP(hipGetLastError());
  return DAIC_OK;
}

}  // extern "C"
