// Set-up of the in-edge form used by dense rounds: a renumbering of the
// sources by out-degree and the transposed CSR sorted by (target, renumbered
// source), built on the device with radix sorts, plus the edge blocks of the
// streamed pull.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include "daic_device.h"
#include "daic_internal.h"

namespace daic {

namespace {

// key = (~outdeg << 32) | j: ascending order = out-degree descending, ties by id.
__global__ void k_degree_keys(const uint32_t* row, uint64_t n, uint64_t* keys) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = i; j < n; j += st) {
    uint32_t deg = row[j + 1] - row[j];
    keys[j] = ((uint64_t)(~deg) << 32) | j;
  }
}

__global__ void k_perm_from_sorted(const uint64_t* sorted, uint64_t n, uint32_t* perm) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t r = i; r < n; r += st) perm[(uint32_t)sorted[r]] = (uint32_t)r;
}

// key = (target << 32) | perm[source], value = edge, for every edge (rows
// walked by lane groups, hub rows by whole waves).
__global__ __launch_bounds__(256) void k_edge_keys(const uint32_t* __restrict__ row, const uint32_t* __restrict__ col,
                                                   const uint32_t* __restrict__ perm, uint64_t n,
                                                   uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  rows_by_groups<false>(
      row, n, [&](uint64_t, uint32_t e) { return col[e]; },
      [&](uint64_t j, uint32_t e, uint32_t t) {
        keys[e] = ((uint64_t)t << 32) | perm[j];
        vals[e] = e;
        return 0.0;
      },
      [](uint64_t, double) {});
}

// srcT from the sorted keys, and the in-edge offsets: rowT[t] = first position
// whose target is >= t.
__global__ void k_split_sorted(const uint64_t* keys, uint64_t m, uint64_t n, uint32_t* srcT, uint32_t* rowT) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t p = i; p < m; p += st) {
    uint64_t k = keys[p];
    srcT[p] = (uint32_t)k;
    uint64_t t = k >> 32;
    uint64_t prev = p == 0 ? 0 : (keys[p - 1] >> 32) + 1;
    if (p == 0) prev = 0;
    for (uint64_t u = prev; u <= t; ++u) rowT[u] = (uint32_t)p;
  }
  if (i == 0) {
    uint64_t last = m == 0 ? 0 : (keys[m - 1] >> 32) + 1;
    for (uint64_t u = last; u <= n; ++u) rowT[u] = (uint32_t)m;
  }
}

uint32_t grid(uint64_t count) {
  uint64_t g = (count + 255) / 256;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g, 8192));
}

}  // namespace

void stream_blocks(const uint32_t* rt, uint64_t t_begin, uint64_t t_end, std::vector<uint32_t>& bt,
                   std::vector<uint32_t>& be, std::vector<uint32_t>& bn, bool cover_all) {
  for (uint64_t t = t_begin; t < t_end;) {
    const uint64_t deg = rt[t + 1] - rt[t];
    if (deg == 0 && !cover_all) {
      ++t;
      continue;
    }
    if (deg > kStreamEdges) {
      for (uint64_t o = 0; o < deg; o += kStreamEdges) {
        bt.push_back((uint32_t)t);
        be.push_back((uint32_t)(rt[t] + o));
        bn.push_back(1);
      }
      ++t;
      continue;
    }
    uint64_t t1 = t + 1;
    while (t1 < t_end && t1 - t < kStreamRows && (uint64_t)rt[t1 + 1] - rt[t] <= kStreamEdges) ++t1;
    bt.push_back((uint32_t)t);
    be.push_back(rt[t]);
    bn.push_back((uint32_t)(t1 - t));
    t = t1;
  }
}

void pull_release(daic_graph* g) {
  PullGraph& p = g->pull;
  for (void* q : {(void*)p.perm, p.rowT, (void*)p.srcT, (void*)p.eidT, (void*)p.sb_t, (void*)p.sb_e, (void*)p.sb_n,
                  (void*)p.sb_g, (void*)p.g_np, (void*)p.g_first})
    if (q) (void)hipFree(q);
  p = PullGraph();
}

daic_status pull_prepare(daic_graph* g, hipStream_t s) {
  PullGraph& P = g->pull;
  if (P.ready) return DAIC_OK;
  const GraphDev& d = g->dev;
  const uint64_t n = d.n, m = d.m;
  if (!d.row32 || m > 0x7FFFFFFFull || n > 0x7FFFFFFFull)
    return fail(DAIC_E_UNSUPPORTED, "dense rounds need n, m < 2^31");
  const uint32_t* row = static_cast<const uint32_t*>(d.row);
  uint64_t *k0 = nullptr, *k1 = nullptr;
  uint32_t *v0 = nullptr, *v1 = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  daic_status rc = DAIC_OK;
  auto cleanup = [&]() {
    for (void* q : {(void*)k0, (void*)k1, (void*)v0, (void*)v1, tmp})
      if (q) (void)hipFree(q);
  };
#define PCHK(call)                                                                             \
  do {                                                                                         \
    hipError_t _e = (call);                                                                    \
    if (_e != hipSuccess) {                                                                    \
      cleanup();                                                                               \
      pull_release(g);                                                                         \
      return fail(_e == hipErrorOutOfMemory ? DAIC_E_OOM : DAIC_E_DEVICE, "dense-round set-up: %s: %s", \
                  #call, hipGetErrorString(_e));                                              \
    }                                                                                          \
  } while (0)
  const uint64_t cap = std::max<uint64_t>(std::max(n, m), 1);
  PCHK(hipMalloc(&k0, cap * sizeof(uint64_t)));
  PCHK(hipMalloc(&k1, cap * sizeof(uint64_t)));
  PCHK(hipMalloc(&v0, std::max<uint64_t>(m, 1) * sizeof(uint32_t)));
  PCHK(hipMalloc(&v1, std::max<uint64_t>(m, 1) * sizeof(uint32_t)));
  PCHK(hipMalloc(&P.perm, std::max<uint64_t>(n, 1) * sizeof(uint32_t)));
  PCHK(hipMalloc(&P.rowT, (n + 1) * sizeof(uint32_t)));
  PCHK(hipMalloc(&P.srcT, std::max<uint64_t>(m, 1) * sizeof(uint32_t)));
  PCHK(hipMalloc(&P.eidT, std::max<uint64_t>(m, 1) * sizeof(uint32_t)));

  // 1. renumbering by out-degree
  hipLaunchKernelGGL(k_degree_keys, dim3(grid(n)), dim3(256), 0, s, row, n, k0);
  {
    hipcub::DoubleBuffer<uint64_t> kb(k0, k1);
    size_t need = 0;
    PCHK(hipcub::DeviceRadixSort::SortKeys(nullptr, need, kb, (int)n, 0, 64, s));
    if (need > tmp_bytes) {
      if (tmp) (void)hipFree(tmp);
      tmp = nullptr;
      PCHK(hipMalloc(&tmp, need));
      tmp_bytes = need;
    }
    PCHK(hipcub::DeviceRadixSort::SortKeys(tmp, need, kb, (int)n, 0, 64, s));
    hipLaunchKernelGGL(k_perm_from_sorted, dim3(grid(n)), dim3(256), 0, s, kb.Current(), n, P.perm);
  }
  // 2. in-edges sorted by (target, renumbered source), carrying the edge index
  if (m > 0) {
    hipLaunchKernelGGL(k_edge_keys, dim3(std::max<uint64_t>(1, std::min<uint64_t>((n + 3) / 4, 8192))), dim3(256), 0,
                       s, row, d.col, P.perm, n, k0, v0);
    hipcub::DoubleBuffer<uint64_t> kb(k0, k1);
    hipcub::DoubleBuffer<uint32_t> vb(v0, v1);
    int end_bit = 32;
    while ((1ull << (end_bit - 32)) < n) ++end_bit;
    size_t need = 0;
    PCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, need, kb, vb, (int)m, 0, end_bit, s));
    if (need > tmp_bytes) {
      if (tmp) (void)hipFree(tmp);
      tmp = nullptr;
      PCHK(hipMalloc(&tmp, need));
      tmp_bytes = need;
    }
    PCHK(hipcub::DeviceRadixSort::SortPairs(tmp, need, kb, vb, (int)m, 0, end_bit, s));
    hipLaunchKernelGGL(k_split_sorted, dim3(grid(m)), dim3(256), 0, s, kb.Current(), m, n, P.srcT,
                       static_cast<uint32_t*>(P.rowT));
    PCHK(hipMemcpyAsync(P.eidT, vb.Current(), m * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
  } else {
    hipLaunchKernelGGL(k_split_sorted, dim3(1), dim3(256), 0, s, k0, 0, n, P.srcT, static_cast<uint32_t*>(P.rowT));
  }
  // 3. edge blocks of the streamed pull (built on the host from the offsets)
  std::vector<uint32_t> rt(n + 1);
  PCHK(hipMemcpyAsync(rt.data(), P.rowT, (n + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  PCHK(hipStreamSynchronize(s));
  cleanup();
  k0 = k1 = nullptr;
  v0 = v1 = nullptr;
  tmp = nullptr;
  for (uint64_t t = 0; t < n; ++t) P.n_targets += rt[t + 1] > rt[t] ? 1 : 0;
  // every target is in one block (the fused dense round claims through them)
  std::vector<uint32_t> bt, be, bn;
  stream_blocks(rt.data(), 0, n, bt, be, bn, true);
  be.push_back((uint32_t)m);
  P.sb_count = bt.size();
  // pieces of one cut target form a group; the last piece of a round to
  // finish claims the target
  std::vector<uint32_t> bg(bt.size(), 0xFFFFFFFFu), gnp, gfirst;
  for (size_t b = 0; b < bt.size();) {
    size_t e = b + 1;
    while (e < bt.size() && bn[b] == 1 && bn[e] == 1 && bt[e] == bt[b]) ++e;
    if (e - b > 1) {
      for (size_t k = b; k < e; ++k) bg[k] = (uint32_t)gnp.size();
      gnp.push_back((uint32_t)(e - b));
      gfirst.push_back((uint32_t)b);
      P.n_pieces += e - b;
    }
    b = e;
  }
  P.n_groups = gnp.size();
  {
    // sources are renumbered by out-degree, descending: those with out-edges first
    const uint32_t* rowp = static_cast<const uint32_t*>(d.row);
    std::vector<uint32_t> ro(n + 1);
    PCHK(hipMemcpy(ro.data(), rowp, (n + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost));
    uint64_t ns = 0;
    for (uint64_t j = 0; j < n; ++j) ns += ro[j + 1] > ro[j] ? 1 : 0;
    P.n_src = ns;
  }
  PCHK(hipMalloc(&P.sb_g, std::max<size_t>(bg.size(), 1) * 4));
  PCHK(hipMalloc(&P.g_np, std::max<size_t>(gnp.size(), 1) * 4));
  if (!bg.empty()) PCHK(hipMemcpy(P.sb_g, bg.data(), bg.size() * 4, hipMemcpyHostToDevice));
  if (!gnp.empty()) PCHK(hipMemcpy(P.g_np, gnp.data(), gnp.size() * 4, hipMemcpyHostToDevice));
  PCHK(hipMalloc(&P.g_first, std::max<size_t>(gfirst.size(), 1) * 4));
  if (!gfirst.empty()) PCHK(hipMemcpy(P.g_first, gfirst.data(), gfirst.size() * 4, hipMemcpyHostToDevice));
  PCHK(hipMalloc(&P.sb_t, std::max<size_t>(bt.size(), 1) * 4));
  PCHK(hipMalloc(&P.sb_e, be.size() * 4));
  PCHK(hipMalloc(&P.sb_n, std::max<size_t>(bn.size(), 1) * 4));
  if (!bt.empty()) {
    PCHK(hipMemcpy(P.sb_t, bt.data(), bt.size() * 4, hipMemcpyHostToDevice));
    PCHK(hipMemcpy(P.sb_n, bn.data(), bn.size() * 4, hipMemcpyHostToDevice));
  }
  PCHK(hipMemcpy(P.sb_e, be.data(), be.size() * 4, hipMemcpyHostToDevice));
#undef PCHK
  P.ready = true;
  (void)rc;
  return DAIC_OK;
}

}  // namespace daic
