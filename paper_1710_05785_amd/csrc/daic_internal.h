// Internal declarations shared by the translation units of libdaic.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "daic.h"

namespace daic {

// ---- error handling --------------------------------------------------------
void set_error(const char* fmt, ...);
daic_status fail(daic_status s, const char* fmt, ...);

#define DAIC_HIP(call)                                                                   \
  do {                                                                                   \
    hipError_t _e = (call);                                                              \
    if (_e != hipSuccess)                                                                \
      return ::daic::fail(_e == hipErrorOutOfMemory ? DAIC_E_OOM : DAIC_E_DEVICE,        \
                          "%s failed: %s (%s:%d)", #call, hipGetErrorString(_e), __FILE__, \
                          __LINE__);                                                     \
  } while (0)

// ---- tuning constants --------------------------------------------------------
constexpr int kScanBlock = 256;       // threads per block of the per-vertex kernels
constexpr int kMaxScanBlocks = 2048;  // blocks of the per-vertex kernels (upper bound)
constexpr uint32_t kSmallMaxDeg = 32; // out-degree bound of the small bin
constexpr uint32_t kChunk = 1024;     // edges per item of the large bin
constexpr uint32_t kStreamEdges = 2048; // in-edges per block of the streamed pull
constexpr uint32_t kStreamRows = 1024;  // targets per block of the streamed pull
constexpr uint32_t kMaxSamples = 4096;
constexpr uint32_t kInfU32 = 0xFFFFFFFFu;

// ---- device control block -----------------------------------------------------
// One per problem, in device memory. Written by the round kernels, read by the
// host once per check.
struct Ctl {
  double r;              // residual of the current state
  double eps;            // stop threshold for sum problems
  uint64_t pending;      // number of pending vertices of the current state
  uint64_t rounds;       // rounds that did work
  uint64_t max_rounds;   // absolute round limit
  uint64_t activations;  // vertex updates performed
  uint64_t pushed;       // messages sent
  uint64_t pushed_large; // messages sent from large-bin vertices
  uint64_t round_act;    // the last round's activations, messages, large-bin messages
  uint64_t round_pushed;
  uint64_t round_pushed_large;
  uint64_t n_small;      // items in the small bin this round
  uint64_t n_large;      // items in the large bin this round
  uint32_t done;         // stop rule holds
  uint32_t stop;         // round limit reached
  uint32_t ticket;       // last-block detection
  uint32_t sel_mode;     // 0 all pending; 1 key >= tau; 2 key > tau, or == tau within ties
  uint64_t tau;          // threshold key of this round
  uint64_t ties_left;    // keys equal to tau to take (sel_mode 2)
  uint64_t k_rem;        // radix select: rank still to place
  uint64_t radix_prefix; // radix select: key bits fixed so far
  uint32_t radix_skip;   // radix select: nothing to do (all pending fit)
  uint32_t pull;         // the next round runs as a pull over in-edges (dense round)
  uint32_t last_pull;    // the round just run was a dense round
  uint64_t fuse_base;    // fused dense rounds: round count when buffer A was last published
  // learned scheduling, decided on the device each round
  uint32_t use_score;    // this round ranks by priority x network multiplier (else exact top-k)
  uint32_t l_exact_left; // exact rounds still to run before the network is used again
  uint32_t l_run;        // learned rounds since the last exact round
  uint32_t l_pad;
  double l_r0;           // residual at the start of the round
  uint64_t l_rounds0;    // round count at the start of the round
  double l_gain;         // priority realized by the round's updates (sum over the selected vertices)
  double l_exact_eff;    // the judge's figure for the last exact round
  uint64_t l_fallbacks;  // learned rounds that handed the next rounds back to exact selection
  uint64_t l_exact_rounds;  // rounds of a learned run taken by exact selection
};

// Compile-time identity of a (op, g, state, row) instantiation.
enum StateKind { ST_F64 = 0, ST_F32 = 1, ST_F32K = 2, ST_U32 = 3, ST_I32 = 4, ST_F64MIN = 5 };

struct GraphDev {
  uint64_t n = 0, m = 0;
  const void* row = nullptr;   // uint32 or uint64 row offsets (n+1)
  bool row32 = false;
  const uint32_t* col = nullptr;
  const void* w = nullptr;     // weights as given
  daic_dtype w_type = DAIC_NONE;
};

// Vertex partition of the per-vertex kernels: block b owns vertices
// [b*per_block, min(n, (b+1)*per_block)).
struct Partition {
  uint32_t blocks = 0;
  uint64_t per_block = 0;
};

// Learned scheduler hooks (defined with the scheduler network).
daic_status learned_prepare(daic_problem* p, const daic_sched_model* model, hipStream_t s);
// The multiplier array of learned rounds, and the enqueue of the scoring
// kernel (which returns at once in an exact round of a learned run).
daic_status learned_scores_array(daic_problem* p, const daic_sched_model* model, const float** score);
void learned_scores_enqueue(daic_problem* p, const daic_sched_model* model, hipStream_t s);
// Bumped whenever the network's parameters or feature scales change.
uint64_t learned_model_version(const daic_sched_model* model);
// Builds the in-edge form of g (no-op when built). Needs m < 2^32.
daic_status pull_prepare(daic_graph* g, hipStream_t s);
void pull_release(daic_graph* g);
// Edge blocks of the streamed pull over targets [t_begin, t_end) of the
// in-edge offsets rt: whole targets in id order while a block holds at most
// kStreamEdges in-edges and kStreamRows targets; a target with more in-edges
// is cut into pieces of kStreamEdges. Appends (first target, first in-edge,
// targets covered) per block. Targets without in-edges start no block unless
// cover_all (then every target of the range is in exactly one block, and a
// block may have no in-edges).
void stream_blocks(const uint32_t* rt, uint64_t t_begin, uint64_t t_end, std::vector<uint32_t>& bt,
                   std::vector<uint32_t>& be, std::vector<uint32_t>& bn, bool cover_all);

}  // namespace daic

namespace daic {
// In-edge (transposed) form of a graph for dense rounds, built on first use.
// Sources are renumbered by out-degree (descending, ties by id) so that the
// message bases of high-degree senders share cache lines.
struct PullGraph {
  bool ready = false;
  uint32_t* perm = nullptr;     // perm[j] = rank of vertex j by out-degree
  void* rowT = nullptr;         // in-edge offsets, RowT[n+1]
  uint32_t* srcT = nullptr;     // perm[source] of each in-edge, sorted by (target, perm[source])
  uint32_t* eidT = nullptr;     // original edge index of each in-edge (weighted graphs)
  uint64_t n_targets = 0;         // targets with in-edges
  uint64_t n_src = 0;             // vertices with out-edges: renumbered positions [0, n_src)
  uint32_t* sb_t = nullptr;       // edge blocks of the streamed pull (first target,
  uint32_t* sb_e = nullptr;       //   first in-edge with a closing entry m,
  uint32_t* sb_n = nullptr;       //   targets covered)
  uint64_t sb_count = 0;
  uint32_t* sb_g = nullptr;       // group of a piece of a cut target, else 0xFFFFFFFF
  uint32_t* g_np = nullptr;       // pieces of each group
  uint32_t* g_first = nullptr;    // first block of each group
  uint64_t n_groups = 0;
  uint64_t n_pieces = 0;          // blocks that are pieces of cut targets
};
}  // namespace daic

namespace daic {
// Partition-tiled in-edge form of dense rounds. Targets are cut into
// partitions of 2^tbits consecutive ids (kTileT, or narrower for graphs with
// fewer than 1,024 kTileT-wide partitions, so that a round has enough tiles). Inside a partition the in-edges are
// sorted by (renumbered source, target), so the in-edges one source sends
// into the partition are consecutive: such a run is a "pair" (source,
// partition) whose message base is gathered once. A partition's in-edges are
// cut into tiles (of up to one CU's share of the in-edges for dense rounds, a
// fraction of a block's for sweeps, at least tile_default_edges); a partition
// with one tile is summed and finished by one workgroup, the tiles of a larger
// one store partial sums that a finishing kernel adds in tile order.
constexpr uint32_t kTileT = 16384;     // most targets per partition (local ids fit 14 bits)
constexpr uint32_t kTileE = 196608;    // in-edges per tile by default (smaller graphs: fewer)
constexpr uint32_t kNarrowTW = 2048;   // widest partition of the 256-thread tile workgroups
// resident tile workgroups per CU: one of 1024 threads (128 KiB of LDS), or
// about four of 256 threads (their registers)
inline uint32_t tile_wgs_per_cu(uint32_t lb) { return (1u << lb) > kNarrowTW ? 1u : 4u; }
constexpr uint16_t kPairStart = 0x8000;  // flag of a pair's first in-edge in tloc
// Segments of padding after the tiled per-in-edge arrays (tloc, segpair and
// weights in tile order): zero local targets with no pair start, segment
// pair 0 and weight 0, so a walk's whole step of segments loads in bounds
// with 32-bit unclamped indices.
constexpr uint32_t kTilePadSeg = 32;
struct TileGraph {
  bool ready = false;
  uint32_t tbits = 14;             // partition width 2^tbits (at most kTileT; smaller graphs get narrower ones)
  uint64_t n_part = 0, n_tiles = 0, n_pairs = 0, n_split = 0, n_slots = 0, n_seg = 0;
  uint16_t* tloc = nullptr;        // [m, padded] target - partition base, | kPairStart at a pair's first in-edge
  uint32_t* psrc = nullptr;        // [n_pairs] renumbered source of each pair
  uint32_t* segpair = nullptr;     // [n_seg, padded] pair of the first in-edge of each 64-in-edge segment
  uint32_t* eid = nullptr;         // [m] original edge index (weights in tile order)
  uint32_t* tile_part = nullptr;   // [n_tiles] partition of each tile
  uint32_t* tile_e = nullptr;      // [n_tiles + 1] first in-edge of each tile (tiles are contiguous)
  uint32_t* tile_slot = nullptr;   // [n_tiles] partial-sum slot, or 0xFFFFFFFF (partition of one tile)
  uint32_t* tile_order = nullptr;  // [n_tiles] launch order: largest tiles first (by in-edges, plus the
                                   // targets an unsplit tile finishes), within groups of partitions
  uint32_t* split_part = nullptr;  // [n_split] partitions of several tiles
  uint32_t* split_slot = nullptr;  // [n_split + 1] their first slot (slots of one partition are consecutive)
  // Targets numbered by in-degree octave, highest first, ids ascending within
  // an octave (the layout of fused dense rounds): a partition then holds
  // targets of similar in-degree and nearby ids, so the hub partitions take
  // the senders' in-edges in long pairs (RMAT-24: 72 M pairs instead of 123 M
  // with id ranges). Null for partitions of consecutive ids. The fused rounds
  // keep the state in this numbering.
  uint32_t* tinv = nullptr;        // [n] vertex of each target number
  uint32_t* rowP = nullptr;        // [n + 1] out-edge offsets in target-number order
  uint32_t* permP = nullptr;       // [n] source number of the vertex of each target number
};
daic_status tile_prepare(daic_graph* g, hipStream_t s);
// The same form with targets numbered by in-degree octave (g->tile_r).
daic_status tile_prepare_ranked(daic_graph* g, hipStream_t s);
// The numbering of targets by in-degree octave within blocks of `block`
// consecutive ids (a block's targets keep its id range): trank (vertex ->
// number) and, per number, its vertex (tinv), out-edge offsets (rowP, n + 1)
// and source number perm[vertex] (permP); device arrays the caller frees.
daic_status rank_targets(const daic_graph* g, const uint32_t* perm, uint64_t block, uint32_t** trank,
                         uint32_t** tinv, uint32_t** rowP, uint32_t** permP, hipStream_t s);
// dst[r] = src[tinv[r]] (gather) or dst[tinv[r]] = src[r] (scatter) for r < n,
// elements of 4 or 8 bytes, enqueued on s.
void perm_gather(const void* src, void* dst, size_t elem, const uint32_t* tinv, uint64_t n, hipStream_t s);
void perm_scatter(const void* src, void* dst, size_t elem, const uint32_t* tinv, uint64_t n, hipStream_t s);
// Entries of the per-in-edge arrays in tile order with their padding.
inline uint64_t tile_padded_edges(const TileGraph& T) { return (T.n_seg + kTilePadSeg) * 64; }
// The tiled kernels index in-edges (with the padding) in 32 bits; larger
// graphs keep the streamed (sum) or push-only (min/max) rounds.
inline bool tile_fits(uint64_t m) { return m + 64ull * (kTilePadSeg + 1) <= 0xFFFFFFFFull; }
// The tiled form of g's in-edges with sources numbered by perm (a device
// array, perm[j] = number of vertex j) and partitions of 2^lb targets
// (8 <= lb <= 14), tiles of at most max_edges in-edges (when nonzero; else
// tile_default_edges); with share_div nonzero, of at most 1/share_div of
// their group's in-edges (and max_edges when nonzero), into T; tile_order
// sorts the tiles within each group of group_parts consecutive partitions
// (all of them when 0); with trank (a device array, or null for target
// ids), targets are placed by trank[t] instead of t; tile_free releases it.
daic_status tile_build(const GraphDev& d, const uint32_t* perm, uint32_t lb, uint64_t max_edges,
                       uint64_t group_parts, uint32_t share_div, TileGraph& T, hipStream_t s,
                       const uint32_t* trank = nullptr);
void tile_free(TileGraph& T);
uint32_t tile_default_bits(uint64_t n);
uint64_t tile_default_edges(uint64_t n, uint64_t m, uint32_t lb);
void tile_release(daic_graph* g);
}  // namespace daic

struct daic_graph {
  daic::GraphDev dev;
  daic::PullGraph pull;
  daic::TileGraph tile;
  daic::TileGraph tile_r;       // targets numbered by in-degree octave (fused dense rounds)
  void* own_row = nullptr;      // owned allocations (null when borrowed)
  void* own_col = nullptr;
  void* own_w = nullptr;
  void* row32 = nullptr;        // narrowed copy of row_ptr when m < 2^32
  daic::Partition part;
  uint64_t* large_off = nullptr;  // device [blocks+1]: large-bin region start per block
  uint64_t large_cap = 0;
};
