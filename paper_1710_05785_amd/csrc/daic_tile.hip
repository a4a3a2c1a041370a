// Set-up of the partition-tiled in-edge form used by fused dense rounds
// (layout in daic_internal.h): in-edges sorted by (partition of the target,
// renumbered source, target) with a device radix sort, pair flags and pair
// sources from a scan of the flags, and the tile table built on the host from
// the partitions' in-edge counts.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include "daic_device.h"
#include "daic_internal.h"

namespace daic {

namespace {

static_assert(kTileT == 1u << 14, "local target offsets and the pair flag share 16 bits");

uint32_t tgrid(uint64_t count) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((count + 255) / 256, 8192));
}

// key = (partition << (sbits + lb)) | (rank << lb) | local target, value =
// the edge, for every edge (rows walked by lane groups); targets placed by
// their number trank[t] when given.
__global__ __launch_bounds__(256) void k_tile_keys(const uint32_t* __restrict__ row, const uint32_t* __restrict__ col,
                                                   const uint32_t* __restrict__ perm,
                                                   const uint32_t* __restrict__ trank, uint64_t n, uint32_t sbits,
                                                   uint32_t lb, uint64_t* __restrict__ keys,
                                                   uint32_t* __restrict__ vals) {
  rows_by_groups<false>(
      row, n, [&](uint64_t, uint32_t e) { return col[e]; },
      [&](uint64_t j, uint32_t e, uint64_t t0) {
        const uint64_t t = trank ? trank[t0] : t0;
        const uint64_t rank = perm[j];
        keys[e] = ((t >> lb) << (sbits + lb)) | (rank << lb) | (t & ((1ull << lb) - 1));
        vals[e] = e;
        return 0.0;
      },
      [](uint64_t, double) {});
}

// Pair flags (a new (partition, source) run starts), local targets and edge
// indices in sorted order.
__global__ void k_tile_flags(const uint64_t* keys, const uint32_t* vals, uint64_t m, uint32_t lb, uint32_t* flag,
                             uint16_t* tloc, uint32_t* eid) {
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[p];
    const bool start = p == 0 || (keys[p - 1] >> lb) != (k >> lb);
    flag[p] = start ? 1u : 0u;
    tloc[p] = (uint16_t)((k & ((1ull << lb) - 1)) | (start ? kPairStart : 0));
    eid[p] = vals[p];
  }
}

// Pair sources, the pair of each 64-in-edge segment's first in-edge, and the
// first in-edge of every partition.
__global__ void k_tile_pairs(const uint64_t* keys, const uint32_t* flag, const uint32_t* incl, uint64_t m,
                             uint32_t sbits, uint32_t lb, uint64_t n_part, uint32_t* psrc, uint32_t* segpair,
                             uint32_t* pstart) {
  const uint64_t smask = (1ull << sbits) - 1;
  const uint32_t pshift = sbits + lb;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[p];
    if (flag[p]) psrc[incl[p] - 1] = (uint32_t)((k >> lb) & smask);
    if ((p & 63) == 0) segpair[p >> 6] = incl[p] - 1;
    const uint64_t part = k >> pshift;
    const uint64_t prev = p == 0 ? 0 : (keys[p - 1] >> pshift) + 1;
    for (uint64_t q = prev; q <= part; ++q) pstart[q] = (uint32_t)p;
    if (p == m - 1)
      for (uint64_t q = part + 1; q <= n_part; ++q) pstart[q] = (uint32_t)m;
  }
}

// The tile table of a partitioned in-edge order, on the host: pstart[p] is
// the first in-edge of partition p (n_part + 1 entries, non-decreasing).
// Every partition gets at least one tile (its targets are finished by it);
// one with more in-edges than its cap is cut into cap-sized tiles and a
// remainder, which get consecutive slots. The cap is ecap, or with share_div
// 1/share_div of the in-edges of its group of group_parts partitions (at
// least 1,024; under ecap when max_edges is given). The launch order sorts
// the tiles within each group by work, largest first: a tile's in-edges
// plus, for an unsplit partition, about two in-edges' worth per target for
// finishing them.
struct TileTable {
  std::vector<uint32_t> tp, te, ts, sp, ss, order;  // te and ss carry one closing entry
  uint32_t slots = 0;
};

TileTable tile_table(const uint32_t* pstart, uint64_t n_part, uint64_t TW, uint64_t ecap, uint64_t max_edges,
                     uint64_t group_parts, uint32_t share_div) {
  TileTable X;
  const uint64_t gp = group_parts ? group_parts : n_part;
  uint64_t gcap = ecap;  // the cap of the current group
  for (uint64_t p = 0; p < n_part; ++p) {
    if (share_div && p % gp == 0) {
      const uint64_t g1 = std::min<uint64_t>(n_part, p + gp);
      gcap = std::max<uint64_t>(1024, (pstart[g1] - pstart[p]) / share_div);
      if (max_edges) gcap = std::min(gcap, ecap);
    }
    const uint64_t a = pstart[p], b = pstart[p + 1];
    const uint64_t nt = std::max<uint64_t>(1, (b - a + gcap - 1) / gcap);
    if (nt > 1) {
      X.sp.push_back((uint32_t)p);
      X.ss.push_back(X.slots);
    }
    for (uint64_t k = 0; k < nt; ++k) {
      X.tp.push_back((uint32_t)p);
      X.te.push_back((uint32_t)(a + k * gcap));
      X.ts.push_back(nt > 1 ? X.slots++ : 0xFFFFFFFFu);
    }
  }
  X.te.push_back(pstart[n_part]);
  X.ss.push_back(X.slots);
  const uint32_t n_tiles = (uint32_t)X.tp.size();
  X.order.resize(n_tiles);
  for (uint32_t i = 0; i < n_tiles; ++i) X.order[i] = i;
  auto work = [&](uint32_t x) {
    return (uint64_t)(X.te[x + 1] - X.te[x]) + (X.ts[x] == 0xFFFFFFFFu ? 2 * TW : 0);
  };
  for (uint32_t b = 0; b < n_tiles;) {
    uint32_t e = b;
    while (e < n_tiles && X.tp[e] / gp == X.tp[b] / gp) ++e;
    std::stable_sort(X.order.begin() + b, X.order.begin() + e,
                     [&](uint32_t x, uint32_t y) { return work(x) > work(y); });
    b = e;
  }
  return X;
}

// Sort keys of the target numbering: the in-degree's octave, highest first
// (the leading zeros of in-degree + 1), then id (the radix sort is stable
// and the values start in id order). On RMAT-24 octaves gave a 0.49 ms pull,
// exact in-degrees 0.55 ms (as many pairs, but the id order inside an octave
// keeps targets of nearby ids, which share senders, in one partition),
// half-octaves 0.50 ms, quarter-range (powers of 4) 0.53 ms, ids alone 0.63 ms.
// Blocks of `block` ids come first in the key, so a block's targets keep its
// id range (one block of all ids for fused rounds).
__global__ void k_indeg_keys(const uint32_t* rowT, uint64_t n, uint64_t block, uint32_t* key, uint32_t* val) {
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (uint64_t)gridDim.x * blockDim.x) {
    key[j] = (uint32_t)((j / block) << 6) | (uint32_t)__clz(rowT[j + 1] - rowT[j] + 1);
    val[j] = (uint32_t)j;
  }
}

// From the numbering's inverse tinv: the number of each vertex, and per
// number its vertex's out-degree and source number.
__global__ void k_rank_tables(const uint32_t* tinv, const uint32_t* row, const uint32_t* perm, uint64_t n,
                              uint32_t* trank, uint32_t* degP, uint32_t* permP) {
  for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t j = tinv[r];
    trank[j] = (uint32_t)r;
    degP[r] = row[j + 1] - row[j];
    permP[r] = perm[j];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) degP[n] = 0;
}

}  // namespace

void tile_free(TileGraph& t) {
  for (void* q : {(void*)t.tloc, (void*)t.psrc, (void*)t.segpair, (void*)t.eid, (void*)t.tile_part, (void*)t.tile_e,
                  (void*)t.tile_slot, (void*)t.tile_order, (void*)t.split_part, (void*)t.split_slot, (void*)t.tinv,
                  (void*)t.rowP, (void*)t.permP})
    if (q) (void)hipFree(q);
  t = TileGraph();
}

void tile_release(daic_graph* g) {
  tile_free(g->tile);
  tile_free(g->tile_r);
}

// in-edges per tile by default: kTileE, or about two partitions' average for
// smaller graphs (at least 16,384), so that hub partitions split into tiles
// of the common size
uint64_t tile_default_edges(uint64_t n, uint64_t m, uint32_t lb) {
  const uint64_t n_part = std::max<uint64_t>(1, (n + (1ull << lb) - 1) >> lb);
  return std::max<uint64_t>(16384, std::min<uint64_t>(kTileE, 2 * m / n_part));
}

uint32_t tile_default_bits(uint64_t n) {
  // kTileT, narrowed (to at least 1,024) until the graph has 1,024
  // partitions, so that small graphs still give every CU tiles
  uint32_t lb = 14;
  while (lb > 10 && (n >> lb) < 1024) --lb;
  return lb;
}

static void tile_shape(const daic_graph* g, uint32_t* lb_out, uint64_t* max_edges_out);

daic_status tile_prepare(daic_graph* g, hipStream_t s) {
  if (g->tile.ready) return DAIC_OK;
  if (!g->pull.ready) return fail(DAIC_E_INVALID, "tiled rounds need the renumbering of the in-edge form");
  uint32_t lb;
  uint64_t max_edges;
  tile_shape(g, &lb, &max_edges);
  return tile_build(g->dev, g->pull.perm, lb, max_edges, 0, 0, g->tile, s);
}

daic_status rank_targets(const daic_graph* g, const uint32_t* perm, uint64_t block, uint32_t** trank_out,
                         uint32_t** tinv_out, uint32_t** rowP_out, uint32_t** permP_out, hipStream_t s) {
  const uint64_t n = g->dev.n;
  uint32_t *key0 = nullptr, *key1 = nullptr, *val0 = nullptr, *val1 = nullptr, *trank = nullptr, *degP = nullptr;
  uint32_t *tinv = nullptr, *rowP = nullptr, *permP = nullptr;
  void* tmp = nullptr;
  auto release = [&](bool all) {
    for (void* q : {(void*)key0, (void*)key1, (void*)val0, (void*)val1, (void*)degP, tmp})
      if (q) (void)hipFree(q);
    if (all)
      for (void* q : {(void*)trank, (void*)tinv, (void*)rowP, (void*)permP})
        if (q) (void)hipFree(q);
  };
#define RCHK(call)                                                                                          \
  do {                                                                                                      \
    hipError_t _e = (call);                                                                                 \
    if (_e != hipSuccess) {                                                                                 \
      release(true);                                                                                        \
      return fail(_e == hipErrorOutOfMemory ? DAIC_E_OOM : DAIC_E_DEVICE, "target numbering: %s: %s", #call, \
                  hipGetErrorString(_e));                                                                   \
    }                                                                                                       \
  } while (0)
  const uint64_t nn = std::max<uint64_t>(n, 1);
  block = std::max<uint64_t>(block, 1);
  uint32_t end_bit = 6;
  while ((1ull << (end_bit - 6)) < (n + block - 1) / block) ++end_bit;
  if (end_bit > 32) return fail(DAIC_E_INVALID, "target numbering: too many blocks");
  RCHK(hipMalloc(&key0, nn * 4));
  RCHK(hipMalloc(&key1, nn * 4));
  RCHK(hipMalloc(&val0, nn * 4));
  RCHK(hipMalloc(&val1, nn * 4));
  RCHK(hipMalloc(&trank, nn * 4));
  RCHK(hipMalloc(&degP, (n + 1) * 4));
  RCHK(hipMalloc(&rowP, (n + 1) * 4));
  RCHK(hipMalloc(&permP, nn * 4));
  hipLaunchKernelGGL(k_indeg_keys, dim3(tgrid(n)), dim3(256), 0, s, static_cast<const uint32_t*>(g->pull.rowT), n,
                     block, key0, val0);
  hipcub::DoubleBuffer<uint32_t> kb(key0, key1), vb(val0, val1);
  size_t need = 0, need2 = 0;
  RCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, need, kb, vb, (int)n, 0, (int)end_bit, s));
  RCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, need2, degP, rowP, (int)(n + 1), s));
  RCHK(hipMalloc(&tmp, std::max<size_t>(std::max(need, need2), 1)));
  RCHK(hipcub::DeviceRadixSort::SortPairs(tmp, need, kb, vb, (int)n, 0, (int)end_bit, s));
  // the sorted values are the numbering's inverse; keep that buffer
  tinv = vb.Current();
  if (tinv == val0) val0 = nullptr;
  else val1 = nullptr;
  hipLaunchKernelGGL(k_rank_tables, dim3(tgrid(n)), dim3(256), 0, s, tinv, static_cast<const uint32_t*>(g->dev.row),
                     perm, n, trank, degP, permP);
  RCHK(hipcub::DeviceScan::ExclusiveSum(tmp, need2, degP, rowP, (int)(n + 1), s));
  RCHK(hipStreamSynchronize(s));
#undef RCHK
  release(false);
  *trank_out = trank;
  *tinv_out = tinv;
  *rowP_out = rowP;
  *permP_out = permP;
  return DAIC_OK;
}

daic_status tile_prepare_ranked(daic_graph* g, hipStream_t s) {
  TileGraph& T = g->tile_r;
  if (T.ready) return DAIC_OK;
  if (!g->pull.ready) return fail(DAIC_E_INVALID, "tiled rounds need the renumbering of the in-edge form");
  uint32_t *trank = nullptr, *tinv = nullptr, *rowP = nullptr, *permP = nullptr;
  daic_status rc = rank_targets(g, g->pull.perm, g->dev.n, &trank, &tinv, &rowP, &permP, s);
  if (rc) return rc;
  uint32_t lb;
  uint64_t max_edges;
  tile_shape(g, &lb, &max_edges);
  rc = tile_build(g->dev, g->pull.perm, lb, max_edges, 0, 0, T, s, trank);
  (void)hipFree(trank);
  if (rc) {
    for (void* q : {(void*)tinv, (void*)rowP, (void*)permP}) (void)hipFree(q);
    return rc;
  }
  T.tinv = tinv;
  T.rowP = rowP;
  T.permP = permP;
  return DAIC_OK;
}

// Partition width and tile size of dense rounds on g.
static void tile_shape(const daic_graph* g, uint32_t* lb_out, uint64_t* max_edges_out) {
  // tiles of up to one resident workgroup's share of the in-edges (at least
  // the default size): with the largest launched first, the few big tiles of
  // the hub partitions run beside the many whole partitions, and a round has
  // fewer split partitions to finish (RMAT-24, 256 CUs, one workgroup each:
  // 1 M in-edges per tile, pull 0.692 -> 0.635 ms and finish 0.055 ->
  // 0.024 ms against tiles of 196,608; 0.75x or 1.25x that size was 2-4 %
  // slower, 2x was 30 % slower; RMAT-20 SSSP, whose 256-thread workgroups
  // share the CUs, lost 25 % with tiles of one CU's share); DAIC_TILE_EDGES
  // overrides it
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const uint64_t n = g->dev.n, m = g->dev.m;
  // the partition width: RMAT-20 (1,024 partitions of 2^10) took 6.7 ms per
  // PageRank solve and 1.03 / 2.26 ms per SSSP solve (all / sampled), with
  // 2^12: 9.6 ms and 1.03 / 2.23 ms, with 2^14: 12.9 ms and 1.19 / 2.53 ms
  // (DAIC_TILE_BITS overrides it)
  uint32_t lb = tile_default_bits(n);
  if (const char* e = std::getenv("DAIC_TILE_BITS")) lb = (uint32_t)std::max(8ul, std::min(14ul, std::strtoul(e, nullptr, 10)));
  uint64_t max_edges = std::max<uint64_t>(tile_default_edges(n, m, lb), m / ((uint64_t)std::max(cus, 1) * tile_wgs_per_cu(lb)));
  if (const char* e = std::getenv("DAIC_TILE_EDGES")) max_edges = std::strtoull(e, nullptr, 10);
  *lb_out = lb;
  *max_edges_out = max_edges;
}

daic_status tile_build(const GraphDev& d, const uint32_t* perm, uint32_t lb, uint64_t max_edges,
                       uint64_t group_parts, uint32_t share_div, TileGraph& T, hipStream_t s,
                       const uint32_t* trank) {
  if (T.ready) return DAIC_OK;
  if (lb < 8 || lb > 14) return fail(DAIC_E_INVALID, "partition width 2^%u outside 2^8..2^14", lb);
  const uint64_t n = d.n, m = d.m;
  // the sorts and scans below count in int, the walk indexes in 32 bits
  if (!tile_fits(m) || m > 0x7FFFFFFFull)
    return fail(DAIC_E_INVALID, "tiled rounds take fewer than 2^31 in-edges: m = %llu", (unsigned long long)m);
  const uint32_t* row = static_cast<const uint32_t*>(d.row);
  uint32_t sbits = 1;
  while ((1ull << sbits) < n) ++sbits;
  T.tbits = lb;
  const uint64_t TW = 1ull << lb;
  const uint64_t ecap = max_edges ? std::max<uint64_t>(1024, max_edges) : tile_default_edges(n, m, lb);
  T.n_part = (n + TW - 1) / TW;
  const uint32_t pbits_end = sbits + lb + [&] {
    uint32_t b = 1;
    while ((1ull << b) < T.n_part + 1) ++b;
    return b;
  }();
  uint64_t *k0 = nullptr, *k1 = nullptr;
  uint32_t *v0 = nullptr, *v1 = nullptr, *flag = nullptr, *incl = nullptr;  // flag, incl: views of a key buffer
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  auto cleanup = [&]() {
    for (void* q : {(void*)k0, (void*)k1, (void*)v0, (void*)v1, tmp})
      if (q) (void)hipFree(q);
  };
#define TCHK(call)                                                                               \
  do {                                                                                           \
    hipError_t _e = (call);                                                                      \
    if (_e != hipSuccess) {                                                                      \
      cleanup();                                                                                 \
      tile_free(T);                                                                              \
      return fail(_e == hipErrorOutOfMemory ? DAIC_E_OOM : DAIC_E_DEVICE, "tiled-round set-up: %s: %s", #call, \
                  hipGetErrorString(_e));                                                        \
    }                                                                                            \
  } while (0)
  const uint64_t mm = std::max<uint64_t>(m, 1);
  T.n_seg = (m + 63) / 64;
  const uint64_t padded = tile_padded_edges(T);
  TCHK(hipMalloc(&T.tloc, padded * sizeof(uint16_t)));
  TCHK(hipMemsetAsync(T.tloc + m, 0, (padded - m) * sizeof(uint16_t), s));
  TCHK(hipMalloc(&T.eid, mm * sizeof(uint32_t)));
  TCHK(hipMalloc(&T.segpair, (T.n_seg + kTilePadSeg) * sizeof(uint32_t)));
  TCHK(hipMemsetAsync(T.segpair + T.n_seg, 0, kTilePadSeg * sizeof(uint32_t), s));
  std::vector<uint32_t> pstart(T.n_part + 1, 0);
  if (m > 0) {
    TCHK(hipMalloc(&k0, m * sizeof(uint64_t)));
    TCHK(hipMalloc(&k1, m * sizeof(uint64_t)));
    TCHK(hipMalloc(&v0, m * sizeof(uint32_t)));
    TCHK(hipMalloc(&v1, m * sizeof(uint32_t)));
    hipLaunchKernelGGL(k_tile_keys, dim3(std::max<uint64_t>(1, std::min<uint64_t>((n + 3) / 4, 8192))), dim3(256), 0,
                       s, row, d.col, perm, trank, n, sbits, lb, k0, v0);
    hipcub::DoubleBuffer<uint64_t> kb(k0, k1);
    hipcub::DoubleBuffer<uint32_t> vb(v0, v1);
    size_t need = 0;
    TCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, need, kb, vb, (int)m, 0, (int)pbits_end, s));
    TCHK(hipMalloc(&tmp, need));
    tmp_bytes = need;
    TCHK(hipcub::DeviceRadixSort::SortPairs(tmp, need, kb, vb, (int)m, 0, (int)pbits_end, s));
    // the buffers not holding the sorted data take the flags and their scan
    flag = kb.Current() == k0 ? reinterpret_cast<uint32_t*>(k1) : reinterpret_cast<uint32_t*>(k0);
    incl = flag + m;  // the other half of the 8-byte-per-edge buffer
    hipLaunchKernelGGL(k_tile_flags, dim3(tgrid(m)), dim3(256), 0, s, kb.Current(), vb.Current(), m, lb, flag,
                       T.tloc, T.eid);
    size_t need2 = 0;
    TCHK(hipcub::DeviceScan::InclusiveSum(nullptr, need2, flag, incl, (int)m, s));
    if (need2 > tmp_bytes) {
      (void)hipFree(tmp);
      tmp = nullptr;
      TCHK(hipMalloc(&tmp, need2));
      tmp_bytes = need2;
    }
    TCHK(hipcub::DeviceScan::InclusiveSum(tmp, need2, flag, incl, (int)m, s));
    uint32_t npairs = 0;
    TCHK(hipMemcpyAsync(&npairs, incl + (m - 1), 4, hipMemcpyDeviceToHost, s));
    TCHK(hipStreamSynchronize(s));
    T.n_pairs = npairs;
    TCHK(hipMalloc(&T.psrc, std::max<uint64_t>(npairs, 1) * sizeof(uint32_t)));
    uint32_t* dpstart = v0 == vb.Current() ? v1 : v0;  // the free value buffer holds m entries
    uint32_t* own_pstart = nullptr;
    if (T.n_part + 1 > m) {
      TCHK(hipMalloc(&own_pstart, (T.n_part + 1) * sizeof(uint32_t)));
      dpstart = own_pstart;
    }
    hipLaunchKernelGGL(k_tile_pairs, dim3(tgrid(m)), dim3(256), 0, s, kb.Current(), flag, incl, m, sbits, lb,
                       T.n_part, T.psrc, T.segpair, dpstart);
    hipError_t e = hipMemcpyAsync(pstart.data(), dpstart, (T.n_part + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (own_pstart) (void)hipFree(own_pstart);
    TCHK(e);
  } else {
    TCHK(hipMalloc(&T.psrc, sizeof(uint32_t)));
  }
  cleanup();
  k0 = k1 = nullptr;
  v0 = v1 = nullptr;
  tmp = nullptr;
  // the tile table and its launch order: largest tiles first, so that the
  // last workgroups of a round are small ones and its tail is short (RMAT-24
  // pull 0.758 -> 0.692 ms); sweeps sort within each block
  const TileTable X = tile_table(pstart.data(), T.n_part, TW, ecap, max_edges, group_parts, share_div);
  const std::vector<uint32_t>&tp = X.tp, &te = X.te, &ts = X.ts, &sp = X.sp, &ss = X.ss, &order = X.order;
  T.n_tiles = tp.size();
  T.n_split = sp.size();
  T.n_slots = X.slots;
  TCHK(hipMalloc(&T.tile_part, tp.size() * 4));
  TCHK(hipMalloc(&T.tile_e, te.size() * 4));
  TCHK(hipMalloc(&T.tile_slot, ts.size() * 4));
  TCHK(hipMalloc(&T.split_part, std::max<size_t>(sp.size(), 1) * 4));
  TCHK(hipMalloc(&T.split_slot, ss.size() * 4));
  TCHK(hipMemcpy(T.tile_part, tp.data(), tp.size() * 4, hipMemcpyHostToDevice));
  TCHK(hipMemcpy(T.tile_e, te.data(), te.size() * 4, hipMemcpyHostToDevice));
  TCHK(hipMemcpy(T.tile_slot, ts.data(), ts.size() * 4, hipMemcpyHostToDevice));
  if (!sp.empty()) TCHK(hipMemcpy(T.split_part, sp.data(), sp.size() * 4, hipMemcpyHostToDevice));
  TCHK(hipMemcpy(T.split_slot, ss.data(), ss.size() * 4, hipMemcpyHostToDevice));
  TCHK(hipMalloc(&T.tile_order, order.size() * 4));
  TCHK(hipMemcpy(T.tile_order, order.data(), order.size() * 4, hipMemcpyHostToDevice));
#undef TCHK
  T.ready = true;
  return DAIC_OK;
}

}  // namespace daic

extern "C" daic_status daic_tile_table(const uint32_t* pstart, uint64_t n_part, uint32_t lb, uint64_t max_edges,
                                       uint64_t group_parts, uint32_t share_div, uint64_t cap, uint32_t* tile_part,
                                       uint32_t* tile_e, uint32_t* tile_slot, uint32_t* order, uint64_t* n_tiles,
                                       uint64_t* n_split, uint64_t* n_slots) {
  using namespace daic;
  if (!pstart || !n_tiles || !n_split || !n_slots) return fail(DAIC_E_INVALID, "null argument");
  if (n_part == 0) return fail(DAIC_E_INVALID, "n_part must be at least 1");
  if (lb < 8 || lb > 14) return fail(DAIC_E_INVALID, "partition width 2^%u outside 2^8..2^14", lb);
  if (!max_edges && !share_div) return fail(DAIC_E_INVALID, "give max_edges or share_div");
  for (uint64_t p = 0; p < n_part; ++p)
    if (pstart[p + 1] < pstart[p]) return fail(DAIC_E_INVALID, "pstart decreases at %llu", (unsigned long long)p);
  if (pstart[n_part] > 0x7FFFFFFFu) return fail(DAIC_E_INVALID, "at most 2^31 - 1 in-edges");
  const uint64_t ecap = max_edges ? std::max<uint64_t>(1024, max_edges) : ~0ull;
  const TileTable X = tile_table(pstart, n_part, 1ull << lb, ecap, max_edges, group_parts, share_div);
  *n_tiles = X.tp.size();
  *n_split = X.sp.size();
  *n_slots = X.slots;
  if (cap < X.tp.size() + 1) return fail(DAIC_E_INVALID, "output capacity %llu below n_tiles + 1 = %llu",
                                         (unsigned long long)cap, (unsigned long long)(X.tp.size() + 1));
  if (!tile_part || !tile_e || !tile_slot || !order) return fail(DAIC_E_INVALID, "null output array");
  std::copy(X.tp.begin(), X.tp.end(), tile_part);
  std::copy(X.te.begin(), X.te.end(), tile_e);
  std::copy(X.ts.begin(), X.ts.end(), tile_slot);
  std::copy(X.order.begin(), X.order.end(), order);
  return DAIC_OK;
}
