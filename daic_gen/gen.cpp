// Seeded synthetic graph and input generators.
//
// This file builds inputs only: CSR graphs, edge weights, seed sets and plain
// uniform draws. It holds none of the solver arithmetic (no ⊕, no g, no
// priorities) and is shared by the CPU oracle and the GPU library alike.
//
// Every random draw is a pure function of (seed, counter), so the output does
// not depend on the number of threads. The mixing function is the 64-bit
// finalizer of SplitMix64 (Steele, Lea and Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014).
//
// Workload shapes follow the paper's evaluation (Sec. 6.1.2): power-law
// graphs with log-normal degrees, weighted variants with integer or
// log-normal weights; RMAT (Chakrabarti, Zhan, Faloutsos 2004) stands in for
// the paper's 100M-2B node synthetic graphs at one-GPU scale.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// Draw number `ctr` of stream `seed`.
inline uint64_t draw(uint64_t seed, uint64_t ctr) {
  return mix64(mix64(seed + 0x9e3779b97f4a7c15ULL) ^ (ctr * 0x9e3779b97f4a7c15ULL + 0x632be59bd9b4e019ULL));
}

// Uniform double in [0, 1) from the top 53 bits.
inline double unif(uint64_t seed, uint64_t ctr) {
  return (double)(draw(seed, ctr) >> 11) * (1.0 / 9007199254740992.0);
}

// Standard normal by the Box-Muller transform from draws 2*i and 2*i+1.
inline double normal(uint64_t seed, uint64_t i) {
  double u1 = unif(seed, 2 * i);
  double u2 = unif(seed, 2 * i + 1);
  if (u1 < 1e-300) u1 = 1e-300;
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586476925 * u2);
}

// Build a CSR (rows sorted ascending) from an edge list given as (src, dst)
// arrays. row_ptr has n+1 entries, col has m entries.
void edges_to_csr(uint64_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                  uint64_t* row_ptr, uint32_t* col) {
  std::vector<std::atomic<uint64_t>> cnt(n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)n; ++i) cnt[i].store(0, std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < (int64_t)m; ++e) cnt[src[e]].fetch_add(1, std::memory_order_relaxed);
  row_ptr[0] = 0;
  for (uint64_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + cnt[i].load(std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)n; ++i) cnt[i].store(row_ptr[i], std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < (int64_t)m; ++e) {
    uint64_t p = cnt[src[e]].fetch_add(1, std::memory_order_relaxed);
    col[p] = dst[e];
  }
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < (int64_t)n; ++i) std::sort(col + row_ptr[i], col + row_ptr[i + 1]);
}

}  // namespace

extern "C" {

// Raw uniform 64-bit draws: out[i] = draw(seed, first + i).
void gen_draw_u64(uint64_t seed, uint64_t first, uint64_t count, uint64_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)count; ++i) out[i] = draw(seed, first + (uint64_t)i);
}

// Integer weights uniform on {lo..hi}: out[i] = lo + draw(seed, i) mod (hi-lo+1).
void gen_uniform_u32(uint64_t seed, uint64_t count, uint32_t lo, uint32_t hi, uint32_t* out) {
  uint64_t span = (uint64_t)hi - lo + 1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)count; ++i) out[i] = lo + (uint32_t)(draw(seed, (uint64_t)i) % span);
}

// Log-normal doubles exp(mu + sigma*Z).
void gen_lognormal_f64(uint64_t seed, uint64_t count, double mu, double sigma, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)count; ++i) out[i] = std::exp(mu + sigma * normal(seed, (uint64_t)i));
}

// RMAT edge list of m = edgefactor * 2^scale edges, no noise and no vertex
// permutation, duplicates and self-loops kept, turned into a CSR whose rows
// are sorted ascending. Quadrant probabilities a, b, c and d = 1-a-b-c.
// row_ptr: n+1 entries (n = 2^scale); col: m entries. Returns 0 on success.
int gen_rmat(uint32_t scale, uint64_t edgefactor, double a, double b, double c, uint64_t seed,
             uint64_t* row_ptr, uint32_t* col) {
  if (scale == 0 || scale > 31) return -1;
  const uint64_t n = 1ULL << scale;
  const uint64_t m = edgefactor * n;
  std::vector<uint32_t> src(m), dst(m);
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < (int64_t)m; ++e) {
    uint32_t s = 0, d = 0;
    for (uint32_t l = 0; l < scale; ++l) {
      double u = unif(seed, (uint64_t)e * 64 + l);
      uint32_t bit = 1u << (scale - 1 - l);
      if (u < a) {
      } else if (u < ab) {
        d |= bit;
      } else if (u < abc) {
        s |= bit;
      } else {
        s |= bit;
        d |= bit;
      }
    }
    src[e] = s;
    dst[e] = d;
  }
  edges_to_csr(n, m, src.data(), dst.data(), row_ptr, col);
  return 0;
}

// Out-degrees of the directed power-law graph: outdeg_j = min(cap, n-1,
// floor(exp(mu + sigma*Z_j))). Returns m.
uint64_t gen_lognormal_outdeg(uint64_t n, double mu, double sigma, uint64_t cap, uint64_t seed,
                              uint64_t* outdeg) {
  uint64_t m = 0;
  for (uint64_t j = 0; j < n; ++j) {
    double x = std::floor(std::exp(mu + sigma * normal(seed, j)));
    uint64_t dg = x < 0 ? 0 : (x > (double)cap ? cap : (uint64_t)x);
    if (dg > n - 1) dg = n - 1;
    outdeg[j] = dg;
    m += dg;
  }
  return m;
}

// Directed power-law graph: source j draws outdeg[j] distinct targets k != j,
// one after another, with probability proportional to (current in-degree of
// k) + 1 (preferential attachment by in-degree). Sources are processed in
// id order. row_ptr must already hold the prefix sum of outdeg; col receives
// m entries, rows sorted ascending.
void gen_pref_targets(uint64_t n, const uint64_t* row_ptr, uint64_t seed, uint32_t* col) {
  // Fenwick tree over weights indeg_k + 1 (1-based internally).
  std::vector<uint64_t> fw(n + 1, 0);
  auto fw_add = [&](uint64_t i, uint64_t v) {
    for (uint64_t x = i + 1; x <= n; x += x & (~x + 1)) fw[x] += v;
  };
  for (uint64_t i = 0; i < n; ++i) fw_add(i, 1);
  uint64_t total = n;
  uint64_t logn = 1;
  while ((1ULL << logn) <= n) ++logn;
  uint64_t ctr = 0;
  std::vector<uint32_t> row;
  for (uint64_t j = 0; j < n; ++j) {
    uint64_t want = row_ptr[j + 1] - row_ptr[j];
    row.clear();
    while (row.size() < want) {
      uint64_t target = draw(seed, ctr++) % total;  // position in [0, total)
      // Descend: smallest k whose prefix weight exceeds target.
      uint64_t pos = 0, rem = target;
      for (uint64_t step = 1ULL << (logn - 1); step; step >>= 1) {
        if (pos + step <= n && fw[pos + step] <= rem) {
          pos += step;
          rem -= fw[pos];
        }
      }
      uint32_t k = (uint32_t)pos;  // 0-based vertex
      if (k == j) continue;
      if (std::find(row.begin(), row.end(), k) != row.end()) continue;
      row.push_back(k);
      fw_add(k, 1);
      ++total;
    }
    std::sort(row.begin(), row.end());
    std::memcpy(col + row_ptr[j], row.data(), row.size() * sizeof(uint32_t));
  }
}

// In-degree log-normal graph in the style of the paper's synthetic data
// (Sec. 6.1.2): indeg_k = min(n-1, floor(exp(mu + sigma*Z_k))), and the
// in-neighbours of k are drawn uniformly at random (distinct, no self-loop).
// Returns m; when col is null only counts are produced into indeg.
uint64_t gen_indeg_lognormal_count(uint64_t n, double mu, double sigma, uint64_t seed, uint64_t* indeg) {
  uint64_t m = 0;
  for (uint64_t k = 0; k < n; ++k) {
    double x = std::floor(std::exp(mu + sigma * normal(seed, k)));
    uint64_t dg = x < 0 ? 0 : (x > (double)(n - 1) ? n - 1 : (uint64_t)x);
    indeg[k] = dg;
    m += dg;
  }
  return m;
}

// Fills the CSR (by source) of the in-degree log-normal graph whose
// in-degrees were produced by gen_indeg_lognormal_count.
void gen_indeg_lognormal_edges(uint64_t n, const uint64_t* indeg, uint64_t seed, uint64_t* row_ptr,
                               uint32_t* col) {
  uint64_t m = 0;
  for (uint64_t k = 0; k < n; ++k) m += indeg[k];
  std::vector<uint32_t> src(m), dst(m);
  std::vector<uint64_t> off(n + 1, 0);
  for (uint64_t k = 0; k < n; ++k) off[k + 1] = off[k] + indeg[k];
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < (int64_t)n; ++k) {
    std::vector<uint32_t> picked;
    uint64_t ctr = 0;
    uint64_t want = indeg[k];
    uint64_t stream = seed ^ (0xA5A5A5A5ULL + (uint64_t)k * 0x100000001B3ULL);
    while (picked.size() < want) {
      uint32_t s = (uint32_t)(draw(stream, ctr++) % n);
      if (s == (uint32_t)k) continue;
      if (std::find(picked.begin(), picked.end(), s) != picked.end()) continue;
      picked.push_back(s);
    }
    for (uint64_t t = 0; t < want; ++t) {
      src[off[k] + t] = picked[t];
      dst[off[k] + t] = (uint32_t)k;
    }
  }
  edges_to_csr(n, m, src.data(), dst.data(), row_ptr, col);
}

// Personalization seed sets: for each of n_rhs right-hand sides, a count
// k ~ U{1..max_k} and k distinct vertices drawn uniformly from those with
// out-degree > 0. Stream `seed`, right-hand side r uses counters of block
// (rhs_base + r). counts: n_rhs entries; seeds: n_rhs*max_k entries (unused
// slots set to UINT32_MAX). Returns the number of candidate vertices.
uint64_t gen_ppr_seeds(uint64_t n, const uint64_t* row_ptr, uint64_t seed, uint64_t rhs_base,
                       uint32_t n_rhs, uint32_t max_k, uint32_t* counts, uint32_t* seeds) {
  std::vector<uint32_t> cand;
  for (uint64_t j = 0; j < n; ++j)
    if (row_ptr[j + 1] > row_ptr[j]) cand.push_back((uint32_t)j);
  for (uint32_t r = 0; r < n_rhs; ++r) {
    uint64_t blk = (rhs_base + r) << 20;
    uint32_t k = 1 + (uint32_t)(draw(seed, blk) % max_k);
    if (k > cand.size()) k = (uint32_t)cand.size();
    counts[r] = k;
    uint32_t* out = seeds + (uint64_t)r * max_k;
    for (uint32_t t = 0; t < max_k; ++t) out[t] = UINT32_MAX;
    uint32_t got = 0;
    uint64_t ctr = 1;
    while (got < k) {
      uint32_t v = cand[draw(seed, blk + ctr++) % cand.size()];
      bool dup = false;
      for (uint32_t t = 0; t < got; ++t) dup |= (out[t] == v);
      if (!dup) out[got++] = v;
    }
    std::sort(out, out + got);
  }
  return cand.size();
}

}  // extern "C"
