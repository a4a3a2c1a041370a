// Snapshots of a problem's state for checkpoint and resume. At a round
// boundary the state (v, dv) is all that a DAIC computation carries: every
// message sent has been added into the receiver's delta (Eq. async), so a run
// restarted from a saved (v, dv) continues the same computation. This is the
// role of the paper's periodic snapshots of the state table for fault
// tolerance (Sec. 5.1), taken here at the end of a run (daic_run returns with
// every message delivered, also when stopped by max_rounds).
//
// Buffer layout (little-endian, version 1):
//   0  char[8]  "DAICPRB1"
//   8  uint32   version (1)
//   12 uint32   state type (daic_dtype)
//   16 uint64   n
//   24 uint64   m
//   32 uint32   op, 36 uint32 g kind
//   40 double   alpha (scalar)
//   48 uint64   payload bytes
//   56 v [n], dv [n] in the device element type (8 bytes for F64 states,
//      4 otherwise), then the compensation term c [n] (FP32) for F32_KAHAN.
#include <hip/hip_runtime.h>

#include <cstring>

#include "daic_internal.h"
#include "daic_problem.h"

namespace daic {

constexpr char kProbMagic[8] = {'D', 'A', 'I', 'C', 'P', 'R', 'B', '1'};
constexpr uint32_t kProbVersion = 1;
constexpr size_t kProbHeader = 56;

static size_t elem_size(int st) { return (st == ST_F64 || st == ST_F64MIN) ? 8 : 4; }

static uint64_t payload_bytes(const daic_problem* p) {
  const uint64_t n = p->g->dev.n;
  return n * 2 * elem_size(p->st) + (p->st == ST_F32K ? n * 4 : 0);
}

}  // namespace daic

using namespace daic;

extern "C" {

daic_status daic_problem_save(const daic_problem* p, void* buf, size_t* len) {
  if (!p || !len) return fail(DAIC_E_INVALID, "null argument");
  const uint64_t need = kProbHeader + payload_bytes(p);
  if (!buf) {
    *len = need;
    return DAIC_OK;
  }
  if (*len < need) {
    const size_t have = *len;
    *len = need;
    return fail(DAIC_E_INVALID, "buffer of %zu bytes, %llu needed", have, (unsigned long long)need);
  }
  uint8_t* b = static_cast<uint8_t*>(buf);
  const uint32_t ver = kProbVersion, st = (uint32_t)p->state, op = (uint32_t)p->op, gk = (uint32_t)p->gk;
  const uint64_t n = p->g->dev.n, m = p->g->dev.m, pay = payload_bytes(p);
  std::memcpy(b, kProbMagic, 8);
  std::memcpy(b + 8, &ver, 4);
  std::memcpy(b + 12, &st, 4);
  std::memcpy(b + 16, &n, 8);
  std::memcpy(b + 24, &m, 8);
  std::memcpy(b + 32, &op, 4);
  std::memcpy(b + 36, &gk, 4);
  std::memcpy(b + 40, &p->alpha, 8);
  std::memcpy(b + 48, &pay, 8);
  const size_t S = elem_size(p->st);
  uint8_t* d = b + kProbHeader;
  DAIC_HIP(hipDeviceSynchronize());
  if (n) {
    DAIC_HIP(hipMemcpy(d, p->a.v, n * S, hipMemcpyDeviceToHost));
    DAIC_HIP(hipMemcpy(d + n * S, p->a.dv, n * S, hipMemcpyDeviceToHost));
    if (p->st == ST_F32K) DAIC_HIP(hipMemcpy(d + 2 * n * S, p->a.c, n * 4, hipMemcpyDeviceToHost));
  }
  *len = need;
  return DAIC_OK;
}

daic_status daic_problem_load(daic_problem* p, const void* buf, size_t len) {
  if (!p || !buf) return fail(DAIC_E_INVALID, "null argument");
  const uint8_t* b = static_cast<const uint8_t*>(buf);
  if (len < kProbHeader || std::memcmp(b, kProbMagic, 8) != 0) return fail(DAIC_E_INVALID, "not a saved problem state");
  uint32_t ver, st, op, gk;
  uint64_t n, m, pay;
  double alpha;
  std::memcpy(&ver, b + 8, 4);
  std::memcpy(&st, b + 12, 4);
  std::memcpy(&n, b + 16, 8);
  std::memcpy(&m, b + 24, 8);
  std::memcpy(&op, b + 32, 4);
  std::memcpy(&gk, b + 36, 4);
  std::memcpy(&alpha, b + 40, 8);
  std::memcpy(&pay, b + 48, 8);
  if (ver != kProbVersion) return fail(DAIC_E_INVALID, "unsupported state version %u", ver);
  if (st != (uint32_t)p->state || op != (uint32_t)p->op || gk != (uint32_t)p->gk)
    return fail(DAIC_E_INVALID, "saved state belongs to another problem kind (op, g or state type differ)");
  if (n != p->g->dev.n || m != p->g->dev.m) return fail(DAIC_E_INVALID, "saved state belongs to another graph size");
  if (std::memcmp(&alpha, &p->alpha, 8) != 0) return fail(DAIC_E_INVALID, "saved state has another alpha");
  if (pay != payload_bytes(p) || len != kProbHeader + pay) return fail(DAIC_E_INVALID, "state buffer has the wrong size");
  const size_t S = elem_size(p->st);
  const uint8_t* d = b + kProbHeader;
  DAIC_HIP(hipDeviceSynchronize());
  if (n) {
    DAIC_HIP(hipMemcpy(p->a.v, d, n * S, hipMemcpyHostToDevice));
    DAIC_HIP(hipMemcpy(p->a.dv, d + n * S, n * S, hipMemcpyHostToDevice));
    if (p->st == ST_F32K) DAIC_HIP(hipMemcpy(p->a.c, d + 2 * n * S, n * 4, hipMemcpyHostToDevice));
  }
  return DAIC_OK;
}

}  // extern "C"
