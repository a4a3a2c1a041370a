// CPU oracle for delta-based accumulative iterative computation (DAIC).
//
// TEST INFRASTRUCTURE ONLY. This code is plain, slow and meant to be checked
// by eye against the paper (Zhang, Gao, Gao, Wang: "Maiter: An Asynchronous
// Graph Processing Framework for Delta-based Accumulative Iterative
// Computation"). It shares no code with the GPU library: only the seeded
// input generators are common to both. Only the test suite, the smoke check
// and the benchmark's CPU-baseline leg may load it.
//
// Floating point is FP64 throughout. Integer problems use 64-bit arithmetic
// internally and report 32-bit results.
//
// Problem encoding used by every entry point:
//   op    : 0 = sum (+), 1 = min, 2 = max                       (Sec. 3.1, third condition)
//   gkind : 0 = g(x) = a_j x            (source scale; Katz, Sec. 4.2 Table 1)
//           1 = g(x) = a_j w_jk x       (edge scale; Adsorption)
//           2 = g(x) = x + w_jk         (edge add; SSSP)
//           3 = g(x) = x                (copy; connected components)
//           4 = g(x) = a x / outdeg_j   (PageRank, sender's out-degree)
//   alpha : scalar a, or per-vertex a_j when alpha_pv is non-null (kinds 0, 1)
//   CSR   : row_ptr[n+1] (uint64), col[m] (uint32); every entry is one edge,
//           duplicates and self-loops included.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>
#include <omp.h>

namespace {

constexpr uint64_t kInfU32 = 0xFFFFFFFFull;  // infinity of the min problems

// Coefficient of edge e = (j -> k) for the linear (sum) problems: the factor
// with which g_{j,k} scales its argument (Sec. 3.1, first condition).
double edge_coef(int gkind, double alpha, const double* alpha_pv, const double* w, uint64_t j,
                 uint64_t e, uint64_t outdeg_j) {
  double a = alpha_pv ? alpha_pv[j] : alpha;
  switch (gkind) {
    case 0: return a;
    case 1: return a * w[e];
    case 4: return alpha / (double)outdeg_j;
    default: return 0.0;
  }
}

// In-edge lists (CSC) with coefficients, in increasing source order, so that
// every pull sums its terms in one fixed order.
struct InEdges {
  std::vector<uint64_t> ptr;
  std::vector<uint32_t> src;
  std::vector<double> coef;
};

InEdges transpose_sum(uint64_t n, const uint64_t* row_ptr, const uint32_t* col, const double* w,
                      int gkind, double alpha, const double* alpha_pv) {
  InEdges t;
  uint64_t m = row_ptr[n];
  t.ptr.assign(n + 1, 0);
  for (uint64_t e = 0; e < m; ++e) t.ptr[col[e] + 1]++;
  for (uint64_t k = 0; k < n; ++k) t.ptr[k + 1] += t.ptr[k];
  std::vector<uint64_t> fill(t.ptr.begin(), t.ptr.end() - 1);
  t.src.resize(m);
  t.coef.resize(m);
  for (uint64_t j = 0; j < n; ++j) {
    uint64_t deg = row_ptr[j + 1] - row_ptr[j];
    for (uint64_t e = row_ptr[j]; e < row_ptr[j + 1]; ++e) {
      uint64_t p = fill[col[e]]++;
      t.src[p] = (uint32_t)j;
      t.coef[p] = edge_coef(gkind, alpha, alpha_pv, w, j, e, deg);
    }
  }
  return t;
}

// Indexed binary max-heap over vertices keyed by (priority, -vid): the largest
// priority first, ties to the smaller vertex id (Sec. 3.5, priority scheduling).
struct MaxHeap {
  std::vector<uint32_t> heap;   // vertex ids
  std::vector<int64_t> where;   // position in heap, -1 if absent
  std::vector<double> key;
  explicit MaxHeap(uint64_t n) : where(n, -1), key(n, 0.0) {}
  bool above(uint32_t a, uint32_t b) const {
    return key[a] > key[b] || (key[a] == key[b] && a < b);
  }
  void swap_at(size_t i, size_t j) {
    std::swap(heap[i], heap[j]);
    where[heap[i]] = (int64_t)i;
    where[heap[j]] = (int64_t)j;
  }
  void up(size_t i) {
    while (i > 0) {
      size_t p = (i - 1) / 2;
      if (!above(heap[i], heap[p])) break;
      swap_at(i, p);
      i = p;
    }
  }
  void down(size_t i) {
    for (;;) {
      size_t l = 2 * i + 1, r = l + 1, b = i;
      if (l < heap.size() && above(heap[l], heap[b])) b = l;
      if (r < heap.size() && above(heap[r], heap[b])) b = r;
      if (b == i) break;
      swap_at(i, b);
      i = b;
    }
  }
  // Set the key of v; a key of 0 removes v (nothing pending).
  void set(uint32_t v, double k) {
    int64_t pos = where[v];
    if (k <= 0.0) {
      if (pos < 0) return;
      size_t last = heap.size() - 1;
      if ((size_t)pos != last) {
        swap_at((size_t)pos, last);
        heap.pop_back();
        where[v] = -1;
        down((size_t)pos);
        up((size_t)pos);
      } else {
        heap.pop_back();
        where[v] = -1;
      }
      key[v] = 0.0;
      return;
    }
    double old = key[v];
    key[v] = k;
    if (pos < 0) {
      heap.push_back(v);
      where[v] = (int64_t)heap.size() - 1;
      up(heap.size() - 1);
    } else if (k > old || (k == old)) {
      up((size_t)pos);
    } else {
      down((size_t)pos);
    }
  }
  bool empty() const { return heap.empty(); }
  uint32_t top() const { return heap[0]; }
};

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------
// O2. Traditional synchronous iteration (Eq. concurrent written in the form of
// Eq. decompose): v^k_j = c_j + sum_{i->j} coef_ij v^{k-1}_i, pulling over the
// in-edges in FP64 with a fixed term order. The constant c follows from the
// fourth condition (Sec. 3.1): v0 + dv1 = f(v0) = M^T v0 + c, i.e.
// c = v0 + dv1 - M^T v0. Starts from v^0 = v0 and stops once
// sum_j |v^k_j - v^{k-1}_j| <= eps or after max_iter sweeps.
// Returns the number of sweeps; *last_diff receives the final L1 change.
// threads <= 0 means all available threads (the result does not depend on it).
int64_t orc_jacobi_sum(uint64_t n, const uint64_t* row_ptr, const uint32_t* col, const double* w,
                       int gkind, double alpha, const double* alpha_pv, const double* v0,
                       const double* dv1, double eps, int64_t max_iter, int threads, double* v_out,
                       double* last_diff) {
  if (threads > 0) omp_set_num_threads(threads);
  InEdges t = transpose_sum(n, row_ptr, col, w, gkind, alpha, alpha_pv);
  std::vector<double> c(n), cur(v0, v0 + n), nxt(n);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t k = 0; k < (int64_t)n; ++k) {
    double s = 0.0;
    for (uint64_t p = t.ptr[k]; p < t.ptr[k + 1]; ++p) s += t.coef[p] * v0[t.src[p]];
    c[k] = v0[k] + dv1[k] - s;
  }
  int64_t it = 0;
  double diff = std::numeric_limits<double>::infinity();
  while (it < max_iter) {
    diff = 0.0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : diff)
    for (int64_t k = 0; k < (int64_t)n; ++k) {
      double s = 0.0;
      for (uint64_t p = t.ptr[k]; p < t.ptr[k + 1]; ++p) s += t.coef[p] * cur[t.src[p]];
      double nv = c[k] + s;
      diff += std::fabs(nv - cur[k]);
      nxt[k] = nv;
    }
    cur.swap(nxt);
    ++it;
    if (diff <= eps) break;
  }
  std::memcpy(v_out, cur.data(), n * sizeof(double));
  if (last_diff) *last_diff = diff;
  return it;
}

// ---------------------------------------------------------------------------
// O3. Synchronous DAIC (Eq. sync) for the sum problems, in push form:
//   v^k_j = v^{k-1}_j + dv^k_j ;  dv^{k+1}_k = sum_j coef_jk dv^k_j.
// v and dv enter holding (v0, dv1) and leave holding the state after the last
// round. Stops when sum_j |dv_j| <= eps (checked before each round) or after
// max_rounds. Returns the number of rounds run.
int64_t orc_sync_daic_sum(uint64_t n, const uint64_t* row_ptr, const uint32_t* col,
                          const double* w, int gkind, double alpha, const double* alpha_pv,
                          double eps, int64_t max_rounds, double* v, double* dv,
                          double* residual) {
  std::vector<double> nxt(n);
  int64_t k = 0;
  double r = 0.0;
  for (;;) {
    r = 0.0;
    for (uint64_t j = 0; j < n; ++j) r += std::fabs(dv[j]);
    if (r <= eps || k >= max_rounds) break;
    std::fill(nxt.begin(), nxt.end(), 0.0);
    for (uint64_t j = 0; j < n; ++j) {
      v[j] += dv[j];
      uint64_t deg = row_ptr[j + 1] - row_ptr[j];
      for (uint64_t e = row_ptr[j]; e < row_ptr[j + 1]; ++e)
        nxt[col[e]] += edge_coef(gkind, alpha, alpha_pv, w, j, e, deg) * dv[j];
    }
    std::memcpy(dv, nxt.data(), n * sizeof(double));
    ++k;
  }
  if (residual) *residual = r;
  return k;
}

// ---------------------------------------------------------------------------
// O4. Asynchronous DAIC (Eq. async), one update at a time on a single thread.
//   update of j:  delta = dv_j; dv_j = identity; v_j = v_j (+) delta;
//                 for every out-edge (j,k): dv_k = dv_k (+) g_jk(delta),
//                 a message equal to the identity being skipped.
// The receive is applied at once (no transmission delay, Sec. 3.4).
//   sched 0: priority scheduling, largest |v_j (+) dv_j - v_j| first, ties to
//            the smaller id (Sec. 3.5; SSSP priority d_j - min(d_j, dd_j)).
//   sched 1: round-robin, sweeping ids 0..n-1 and updating each pending vertex
//            (Sec. 5.1, scheduling within the update thread).
//   sched 2: the synchronous update sequence of Sec. 3.4 (every vertex once per
//            subsequence, in id order), counting every visit as an update, so
//            that max_updates = k n runs exactly k subsequences.
// Sum problems use FP64 v/dv (v_f64, dv_f64) and stop when sum_j |dv_j| <= eps.
// Min problems use uint32 v/dv (v_u32, dv_u32; 0xFFFFFFFF = infinity) with
// saturating g(x) = x + w; max problems use int32 v/dv (v_i32, dv_i32); both
// stop when no vertex is pending. Every problem also stops after max_updates
// updates. Returns the number of updates performed; *residual receives the
// final sum of |dv| (sum) or the number of pending vertices (min/max).
// trace (nullable, length trace_len): progress metric sum_j v_j after update
// number (i+1)*trace_every, for the update-count experiments (Sec. 6.3).
int64_t orc_async(uint64_t n, const uint64_t* row_ptr, const uint32_t* col, const double* w_f64,
                  const uint32_t* w_u32, int op, int gkind, double alpha, const double* alpha_pv,
                  int sched, double eps, int64_t max_updates, double* v_f64, double* dv_f64,
                  uint32_t* v_u32, uint32_t* dv_u32, int32_t* v_i32, int32_t* dv_i32,
                  double* residual, double* trace, int64_t trace_len, int64_t trace_every) {
  auto pending_prio = [&](uint64_t j) -> double {
    if (op == 0) return std::fabs(dv_f64[j]);
    if (op == 1) {
      uint64_t a = v_u32[j], b = dv_u32[j];
      uint64_t mn = std::min(a, b);
      if (a == kInfU32) return mn < kInfU32 ? (double)kInfU32 : 0.0;
      return (double)(a - mn);
    }
    int64_t a = v_i32[j], b = dv_i32[j];
    return (double)(std::max(a, b) - a);
  };
  auto progress = [&]() -> double {
    double s = 0.0;
    for (uint64_t j = 0; j < n; ++j)
      s += op == 0 ? v_f64[j] : (op == 1 ? (double)v_u32[j] : (double)v_i32[j]);
    return s;
  };
  // Exact residual for the sum problems, recomputed from scratch.
  auto exact_r = [&]() -> double {
    double s = 0.0;
    for (uint64_t j = 0; j < n; ++j) s += std::fabs(dv_f64[j]);
    return s;
  };

  MaxHeap heap(sched == 0 ? n : 0);
  uint64_t pending = 0;
  std::vector<char> is_pending(n, 0);
  for (uint64_t j = 0; j < n; ++j) {
    double p = pending_prio(j);
    if (p > 0) {
      is_pending[j] = 1;
      ++pending;
      if (sched == 0) heap.set((uint32_t)j, p);
    }
  }
  long double r_run = op == 0 ? (long double)exact_r() : 0.0L;
  int64_t updates = 0;
  int64_t traced = 0;
  uint64_t rr_next = 0;

  auto done = [&]() -> bool {
    if (updates >= max_updates) return true;
    if (pending == 0 && sched != 2) return true;
    if (pending == 0 && sched == 2) return updates % (int64_t)(n ? n : 1) == 0;
    if (op == 0 && r_run <= (long double)eps) {
      r_run = exact_r();
      return r_run <= (long double)eps;
    }
    return false;
  };

  // Apply a message to dv_k, keeping the pending set, heap and residual.
  auto receive = [&](uint64_t k, double mf, uint64_t mu, int64_t mi) {
    if (op == 0) {
      double before = dv_f64[k];
      dv_f64[k] = before + mf;
      r_run += (long double)std::fabs(dv_f64[k]) - (long double)std::fabs(before);
    } else if (op == 1) {
      if (mu < dv_u32[k]) dv_u32[k] = (uint32_t)mu;
    } else {
      if (mi > dv_i32[k]) dv_i32[k] = (int32_t)mi;
    }
    double p = pending_prio(k);
    if (p > 0 && !is_pending[k]) { is_pending[k] = 1; ++pending; }
    if (p <= 0 && is_pending[k]) { is_pending[k] = 0; --pending; }
    if (sched == 0) heap.set((uint32_t)k, p);
  };

  while (!done()) {
    uint64_t j;
    if (sched == 0) {
      j = heap.top();
    } else if (sched == 1) {
      while (!is_pending[rr_next]) rr_next = (rr_next + 1) % n;
      j = rr_next;
      rr_next = (rr_next + 1) % n;
    } else {
      j = rr_next;
      rr_next = (rr_next + 1) % n;
      if (!is_pending[j]) {  // nothing pending here: the visit changes nothing
        ++updates;
        continue;
      }
    }
    uint64_t deg = row_ptr[j + 1] - row_ptr[j];
    if (op == 0) {
      double delta = dv_f64[j];
      dv_f64[j] = 0.0;
      r_run -= (long double)std::fabs(delta);
      v_f64[j] += delta;
      is_pending[j] = 0;
      --pending;
      if (sched == 0) heap.set((uint32_t)j, 0.0);
      for (uint64_t e = row_ptr[j]; e < row_ptr[j + 1]; ++e) {
        double msg = edge_coef(gkind, alpha, alpha_pv, w_f64, j, e, deg) * delta;
        if (msg != 0.0) receive(col[e], msg, 0, 0);
      }
    } else if (op == 1) {
      uint64_t delta = dv_u32[j];
      dv_u32[j] = (uint32_t)kInfU32;
      bool improves = delta < v_u32[j];
      if (improves) v_u32[j] = (uint32_t)delta;
      is_pending[j] = 0;
      --pending;
      if (sched == 0) heap.set((uint32_t)j, 0.0);
      if (improves && delta < kInfU32) {
        for (uint64_t e = row_ptr[j]; e < row_ptr[j + 1]; ++e) {
          uint64_t msg = delta + (gkind == 2 ? (uint64_t)w_u32[e] : 0);
          if (msg > kInfU32) msg = kInfU32;
          if (msg < kInfU32) receive(col[e], 0.0, msg, 0);
        }
      }
    } else {
      int64_t delta = dv_i32[j];
      dv_i32[j] = -1;
      bool improves = delta > v_i32[j];
      if (improves) v_i32[j] = (int32_t)delta;
      is_pending[j] = 0;
      --pending;
      if (sched == 0) heap.set((uint32_t)j, 0.0);
      if (improves && delta > -1) {
        for (uint64_t e = row_ptr[j]; e < row_ptr[j + 1]; ++e) receive(col[e], 0.0, 0, delta);
      }
    }
    ++updates;
    if (op == 0 && updates % (int64_t)(n ? n : 1) == 0) r_run = exact_r();
    if (trace && trace_every > 0 && updates % trace_every == 0 && traced < trace_len)
      trace[traced++] = progress();
  }
  if (residual) *residual = op == 0 ? exact_r() : (double)pending;
  return updates;
}

// ---------------------------------------------------------------------------
// O5a. Dijkstra with a binary heap and 64-bit distances: the textbook answer of
// the min problem (SSSP, Sec. 4.2.1). Unreached vertices get 0xFFFFFFFF.
// Returns 0, or -1 when some finite distance does not fit below 2^32 - 1.
int orc_dijkstra(uint64_t n, const uint64_t* row_ptr, const uint32_t* col, const uint32_t* w,
                 uint32_t source, uint32_t* dist_out) {
  const uint64_t INF = std::numeric_limits<uint64_t>::max();
  std::vector<uint64_t> dist(n, INF);
  std::vector<char> done(n, 0);
  using Item = std::pair<uint64_t, uint32_t>;
  std::vector<Item> pq;
  auto cmp = [](const Item& a, const Item& b) { return a.first > b.first; };
  dist[source] = 0;
  pq.push_back({0, source});
  while (!pq.empty()) {
    std::pop_heap(pq.begin(), pq.end(), cmp);
    Item it = pq.back();
    pq.pop_back();
    uint32_t u = it.second;
    if (done[u]) continue;
    done[u] = 1;
    for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      uint64_t nd = dist[u] + w[e];
      if (nd < dist[col[e]]) {
        dist[col[e]] = nd;
        pq.push_back({nd, col[e]});
        std::push_heap(pq.begin(), pq.end(), cmp);
      }
    }
  }
  int rc = 0;
  for (uint64_t j = 0; j < n; ++j) {
    if (dist[j] == INF) {
      dist_out[j] = (uint32_t)kInfU32;
    } else if (dist[j] >= kInfU32) {
      rc = -1;
      dist_out[j] = (uint32_t)kInfU32;
    } else {
      dist_out[j] = (uint32_t)dist[j];
    }
  }
  return rc;
}

// ---------------------------------------------------------------------------
// O5b. Max-label reachability: label_j = max({i : i reaches j} U {j}), the
// fixed point of the max problem with g(x) = x, v0 = -1, dv1_j = j
// (connected components, Table 1). Breadth-first search from every vertex in
// descending id order, not entering vertices already labelled: whatever such a
// vertex reaches was already reached from a larger id.
void orc_maxlabel(uint64_t n, const uint64_t* row_ptr, const uint32_t* col, int32_t* label) {
  for (uint64_t j = 0; j < n; ++j) label[j] = -1;
  std::vector<uint32_t> queue;
  for (int64_t s = (int64_t)n - 1; s >= 0; --s) {
    if (label[s] >= 0) continue;
    label[s] = (int32_t)s;
    queue.clear();
    queue.push_back((uint32_t)s);
    for (size_t h = 0; h < queue.size(); ++h) {
      uint32_t u = queue[h];
      for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
        uint32_t k = col[e];
        if (label[k] < 0) {
          label[k] = (int32_t)s;
          queue.push_back(k);
        }
      }
    }
  }
}

}  // extern "C"
